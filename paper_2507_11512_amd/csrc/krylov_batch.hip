// Batched instances of the Krylov passes (K = 2, 4, 8 interleaved
// right-hand sides): the first GEMVT h1 = Q^T w, and the two fused CGS2
// update passes.  The kernel templates are those of the single solve
// (krylov_device.hpp); basis counts are bucketed in steps of 8 columns.
#include "krylov_device.hpp"

#include <stdexcept>
#include <type_traits>

namespace hpgmx {

#define HPGMX_KB8_CASE(N_)                  \
    case N_: {                              \
        constexpr int KB = 8 * N_;          \
        HPGMX_KB_BODY;                      \
    } break;
#define HPGMX_KB8_SWITCH(kb)                                                                   \
    switch (((kb) + 7) / 8) {                                                                  \
        HPGMX_KB8_CASE(1) HPGMX_KB8_CASE(2) HPGMX_KB8_CASE(3) HPGMX_KB8_CASE(4)                \
        HPGMX_KB8_CASE(5) HPGMX_KB8_CASE(6) HPGMX_KB8_CASE(7) HPGMX_KB8_CASE(8)                \
    default: throw std::runtime_error("basis size out of range");                              \
    }

template <typename F> static void with_bk(int K, Prec p, F &&f)
{
    using std::integral_constant;
    const bool d = p == P64;
#define HPGMX_BK(KK)                                                            \
    if (K == KK) {                                                              \
        if (d) return f(integral_constant<int, KK>{}, (double *)nullptr);       \
        return f(integral_constant<int, KK>{}, (float *)nullptr);               \
    }
    HPGMX_BK(2) HPGMX_BK(4) HPGMX_BK(8)
#undef HPGMX_BK
    throw std::runtime_error("unsupported batch width");
}

void batch_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, const void *w, double *partials,
               Ctrl *ctrl, hipStream_t s)
{
    const dim3 gr(red_blocks(M)), bl(kBlock);
    with_bk(K, p, [&](auto kc, auto *tag) {
        constexpr int KK = decltype(kc)::value;
        using T = std::remove_pointer_t<decltype(tag)>;
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_dot<T, KB, KK>), gr, bl, 0, s, M, (const T *)Q, ldq, kb, (const T *)w, partials)
        HPGMX_KB8_SWITCH(kb)
#undef HPGMX_KB_BODY
    });
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)gr.x, kb, K, kFinishH1, ctrl, 0, 0, s);
}

void batch_cgs_dot(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                   Ctrl *ctrl, hipStream_t s)
{
    const dim3 gr(red_blocks(M)), bl(kBlock);
    with_bk(K, p, [&](auto kc, auto *tag) {
        constexpr int KK = decltype(kc)::value;
        using T = std::remove_pointer_t<decltype(tag)>;
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_cgs_dot<T, KB, KK>), gr, bl, 0, s, M, (const T *)Q, ldq, kb, (const T *)w, partials, ctrl)
        HPGMX_KB8_SWITCH(kb)
#undef HPGMX_KB_BODY
    });
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)gr.x, kb, K, kFinishH2, ctrl, 0, 0, s);
}

void batch_cgs_norm(i64 M, int K, Prec p, const void *Q, i64 ldq, int kb, void *w, double *partials,
                    Ctrl *ctrl, int k, int m, hipStream_t s)
{
    const dim3 gr(red_blocks(M)), bl(kBlock);
    with_bk(K, p, [&](auto kc, auto *tag) {
        constexpr int KK = decltype(kc)::value;
        using T = std::remove_pointer_t<decltype(tag)>;
#define HPGMX_KB_BODY \
    hipLaunchKernelGGL((k_cgs_norm<T, KB, KK>), gr, bl, 0, s, M, (const T *)Q, ldq, kb, (T *)w, partials, ctrl)
        HPGMX_KB8_SWITCH(kb)
#undef HPGMX_KB_BODY
    });
    HPGMX_LAUNCH_CHECK();
    launch_finish(partials, (int)gr.x, 1, K, kFinishNormGivens, ctrl, k, m, s);
}

}  // namespace hpgmx
