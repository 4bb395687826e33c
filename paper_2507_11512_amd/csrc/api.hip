// C ABI of hpgmx: handle lifecycle, device memory, the V-cycle and the
// GMRES-IR driver (Alg. 3).  The host side only sequences kernels on the
// handle's stream; all arithmetic runs on the device.
#include "hpgmx_internal.hpp"

#include <cmath>
#include <map>
#include <tuple>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

using namespace hpgmx;

namespace {

struct Error {
    hpgmx_status st;
    std::string msg;
};

[[noreturn]] void fail(hpgmx_status st, const std::string &m) { throw Error{st, m}; }

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) fail(HPGMX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
inline size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct Level {
    Matrix A;
    // work vectors (levels >= 1) per multigrid vector type: [0] double,
    // [1] float, [2] __half, [3] bf16
    void *r[4] = {nullptr, nullptr, nullptr, nullptr};
    void *z[4] = {nullptr, nullptr, nullptr, nullptr};
};

// How the SpMV after a V-cycle shares its work with the V-cycle's last
// level-0 sweep (hpgmx_set_layout spmv_in_sweep).
constexpr int kSpmvPlain = 0;   // one SpMV over all rows
constexpr int kSpmvLast = 1;    // the last colour launch writes its colour's rows
constexpr int kSpmvSplit = 2;   // ... and the three colours before it their partial sums
constexpr int kSpmvSplitSeparate = 3;  // the split sums of kSpmvSplit, all formed by the SpMV
constexpr int kSplitFirst = 2;  // first sweep position with partial sums (see launch_spmv_split)

struct Krylov {
    int m = 0;
    i64 ldq = 0;        // leading dimension of Q (N rounded up, plus a skew)
    void *Q = nullptr;  // (m + 1) columns of ldq
    void *z = nullptr;  // V-cycle output (multigrid vector type), SpMV input
    void *u = nullptr;  // end-of-cycle Q y (Krylov type)
    void *r0 = nullptr; // 16-bit hierarchy: the scaled V-cycle input
    void *part = nullptr;  // partial SpMV sums of the last sweep (Krylov type, N entries)
};

// Index of the multigrid vector type: 0 double, 1 float, 2 __half, 3 bf16.
inline int vt_of(Prec p) { return p == P64 ? 0 : p == P16V ? 2 : p == PB16V ? 3 : 1; }
// Element type of the multigrid vectors of p at the ABI.
inline Prec vprec(Prec p) { return p == P64 ? P64 : mg16(p) ? p : P32; }

// Tile table of the batched stencil kernels: R (right-hand sides per lane)
// per kernel kind and level; 0 = the fixed rule.
struct BatchTune {
    int R[HPGMX_BK_COUNT][kMaxLevels] = {};
    double ms[HPGMX_BK_COUNT][kMaxLevels] = {};
    bool set = false;
};

// State of batched solves with K interleaved right-hand sides.  Vectors are
// [N][K] in the colour-blocked order; those that are gathered from hold
// (N + 1) K entries with row N zero.
struct Batch {
    int K = 0;
    double *b = nullptr, *x = nullptr, *r64 = nullptr;      // FP64, level 0
    Ctrl *ctrl = nullptr;                                    // one per right-hand side
    double *partials = nullptr;                              // kMaxBasis * K columns
    double *host_scal = nullptr;                             // pinned scalar blocks
    void *lr[2][kMaxLevels] = {}, *lz[2][kMaxLevels] = {};  // levels >= 1, [0] double, [1] float
    Krylov kry[2];                                           // per vector type
    void *tmp[2][3] = {};                                    // ABI staging and autotuning
    BatchTune tune[4];                                       // per matrix precision (Prec)
};

}  // namespace

struct hpgmx_ctx {
    hpgmx_problem_desc prob{};  // grid size (beta is unused once `stencil` is set)
    Stencil stencil{};
    bool cols16 = false;        // column format of the hierarchy (hpgmx_set_column_format)
    Layout layout;              // data layout and tile order (hpgmx_set_layout)
    int spmv_mode = kSpmvSplit; // how the V-cycle's last sweep shares the SpMV's work (hpgmx_set_layout)
    hipStream_t stream = nullptr;
    int device = 0;
    bool mg_ready = false;
    bool poisoned = false;
    hpgmx_mg_desc mg{};
    std::vector<Level> lv;

    // memory: bound workspace (bump allocation) or owned hipMalloc blocks
    char *ws_base = nullptr;
    size_t ws_size = 0, ws_used = 0;
    std::vector<void *> owned;

    Krylov kry[kNumPrec];
    double *b_int = nullptr, *x_int = nullptr, *r64 = nullptr;
    double *partials = nullptr;
    Ctrl *ctrl = nullptr;
    double *host_scal = nullptr;   // pinned copies of the Ctrl scalar block (2 slots)
    hipEvent_t ev_scal[2] = {nullptr, nullptr};  // scalar copy of slot s has landed
    void *tmp[4][3] = {};  // ABI staging per multigrid vector type (vt_of)

    // hipGraph replay of inner steps: a private stream (default priority) that
    // can be captured, and one instantiated graph per (dtype, k, m).
    hipStream_t own = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;  // (dtype, k, m, K)

    // batched solves, by interleave width K
    std::map<int, Batch> batches;

    // the last restart cycle of the last single solve, per inner dtype:
    // steps taken and restart length (hpgmx_krylov_cycle_get)
    int last_k[kNumPrec] = {-1, -1, -1, -1, -1, -1};
    int last_m[kNumPrec] = {};

    void drop_graphs()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
    }

    // profiling
    bool prof = false;
    struct Ev {
        hipEvent_t a, b;
        int kernel, level;
    };
    std::vector<Ev> evpool;
    size_t evused = 0;
    double prof_ms[HPGMX_K_COUNT][kMaxLevels] = {};
    long long prof_n[HPGMX_K_COUNT][kMaxLevels] = {};

    std::string err;

    void *dalloc(size_t bytes)
    {
        bytes = round_up(bytes ? bytes : 1);
        if (ws_base) {
            if (ws_used + bytes > ws_size)
                fail(HPGMX_ENOMEM, "bound workspace exhausted (need " + std::to_string(ws_used + bytes) +
                                       " bytes, have " + std::to_string(ws_size) + ")");
            void *p = ws_base + ws_used;
            ws_used += bytes;
            return p;
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(HPGMX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        owned.push_back(p);
        return p;
    }

    // profiling scopes around single launches
    void prof_begin(int kernel, int level)
    {
        if (!prof) return;
        if (evused == evpool.size()) {
            Ev e{};
            hip_check(hipEventCreate(&e.a), "hipEventCreate");
            hip_check(hipEventCreate(&e.b), "hipEventCreate");
            evpool.push_back(e);
        }
        Ev &e = evpool[evused];
        e.kernel = kernel;
        e.level = level;
        hip_check(hipEventRecord(e.a, stream), "hipEventRecord");
    }
    void prof_end()
    {
        if (!prof) return;
        hip_check(hipEventRecord(evpool[evused].b, stream), "hipEventRecord");
        ++evused;
    }
    void prof_collect()
    {
        hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
        for (size_t i = 0; i < evused; ++i) {
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, evpool[i].a, evpool[i].b), "hipEventElapsedTime");
            prof_ms[evpool[i].kernel][evpool[i].level] += ms;
            prof_n[evpool[i].kernel][evpool[i].level] += 1;
        }
        evused = 0;
    }
};

namespace {

struct ProfScope {
    hpgmx_ctx *c;
    ProfScope(hpgmx_ctx *c_, int k, int l) : c(c_) { c->prof_begin(k, l); }
    ~ProfScope() { c->prof_end(); }
};

// A reduction pass and its finish kernel, timed apart: the pass under
// `kernel`, the finish kernel under HPGMX_K_FINISH.
struct PassScope {
    hpgmx_ctx *c;
    static void split(void *a)
    {
        hpgmx_ctx *cc = (hpgmx_ctx *)a;
        cc->prof_end();
        cc->prof_begin(HPGMX_K_FINISH, 0);
    }
    PassScope(hpgmx_ctx *c_, int kernel, int level) : c(c_)
    {
        c->prof_begin(kernel, level);
        if (c->prof) {
            finish_hook = &PassScope::split;
            finish_hook_arg = c;
        }
    }
    ~PassScope()
    {
        finish_hook = nullptr;
        finish_hook_arg = nullptr;
        c->prof_end();
    }
};

// ---- allocation plan ---------------------------------------------------------------------
// Leading dimension of the Krylov basis: N rounded up to 64 elements plus a
// skew of `pad` elements.
i64 krylov_ldq(i64 N, int pad) { return (N + 63) / 64 * 64 + pad; }


void alloc_matrix_prec(hpgmx_ctx *c, Matrix &A, Prec p)
{
    p = matrix_prec(p);
    const size_t N = (size_t)A.g.N, E = (size_t)ell_entries(A.g.N, A.clog2);
    switch (p) {
    case P64:
        if (!A.v64) { A.v64 = (double *)c->dalloc(E * 8); A.d64 = (double *)c->dalloc(N * 8); }
        break;
    case P32:
        if (!A.v32) { A.v32 = (float *)c->dalloc(E * 4); A.d32 = (float *)c->dalloc(N * 4); }
        break;
    case P16:
        if (!A.v16) { A.v16 = (__half *)c->dalloc(E * 2); A.d16 = (__half *)c->dalloc(N * 2); }
        break;
    case PB16:
        if (!A.vb16) { A.vb16 = (bf16 *)c->dalloc(E * 2); A.db16 = (bf16 *)c->dalloc(N * 2); }
        break;
    default: break;  // the 16-bit hierarchies use the P16 / PB16 values
    }
}

bool has_prec(const Matrix &A, Prec p)
{
    switch (matrix_prec(p)) {
    case P64: return A.v64 != nullptr;
    case P32: return A.v32 != nullptr;
    case P16: return A.v16 != nullptr;
    case PB16: return A.vb16 != nullptr;
    default: break;
    }
    return false;
}

// Generates the values of precision p on every level (and the columns once).
void ensure_prec(hpgmx_ctx *c, Prec p)
{
    p = matrix_prec(p);
    for (auto &L : c->lv) {
        if (has_prec(L.A, p)) continue;
        alloc_matrix_prec(c, L.A, p);
        Matrix only = L.A;  // generate just this precision (and nothing else)
        only.col = nullptr;
        if (p != P64) only.v64 = nullptr, only.d64 = nullptr;
        if (p != P32) only.v32 = nullptr, only.d32 = nullptr;
        if (p != P16) only.v16 = nullptr, only.d16 = nullptr;
        if (p != PB16) only.vb16 = nullptr, only.db16 = nullptr;
        launch_generate(only, c->stencil, nullptr, c->stream);
    }
}

// A vector the kernels gather from: N + 1 entries, entry N zero (the
// column of padded ELL slots).
void *gathered_vector(hpgmx_ctx *c, i64 N, Prec p)
{
    char *v = (char *)c->dalloc((size_t)(N + 1) * vec_bytes(p));
    hip_check(hipMemsetAsync(v + (size_t)N * vec_bytes(p), 0, vec_bytes(p), c->stream),
              "hipMemsetAsync");
    return v;
}

// The staging buffers serve every level: re-zero entry N of the level used.
void zero_entry(hpgmx_ctx *c, void *v, i64 N, Prec p)
{
    hip_check(hipMemsetAsync((char *)v + (size_t)N * vec_bytes(p), 0, vec_bytes(p), c->stream),
              "hipMemsetAsync");
}

void ensure_level_vectors(hpgmx_ctx *c, Prec p)
{
    const int vt = vt_of(p);
    for (size_t l = 1; l < c->lv.size(); ++l) {
        Level &L = c->lv[l];
        if (!L.r[vt]) {
            L.r[vt] = gathered_vector(c, L.A.g.N, p);
            L.z[vt] = gathered_vector(c, L.A.g.N, p);
        }
    }
}

void ensure_tmp(hpgmx_ctx *c, Prec p)
{
    const int vt = vt_of(p);
    const size_t N0 = (size_t)c->lv[0].A.g.N;
    for (int i = 0; i < 3; ++i)
        if (!c->tmp[vt][i]) c->tmp[vt][i] = gathered_vector(c, (i64)N0, p);
}

void ensure_common(hpgmx_ctx *c)
{
    if (!c->ctrl) {
        c->ctrl = (Ctrl *)c->dalloc(sizeof(Ctrl));
        hip_check(hipMemsetAsync(c->ctrl, 0, sizeof(Ctrl), c->stream), "hipMemsetAsync");
        c->partials = (double *)c->dalloc((size_t)kMaxRedBlocks * kMaxBasis * 8);
    }
}

void ensure_krylov(hpgmx_ctx *c, Prec p, int m)
{
    ensure_common(c);
    const size_t N0 = (size_t)c->lv[0].A.g.N;
    if (!c->b_int) {
        c->b_int = (double *)c->dalloc(N0 * 8);
        c->x_int = (double *)gathered_vector(c, (i64)N0, P64);
        c->r64 = (double *)c->dalloc(N0 * 8);
    }
    Krylov &K = c->kry[p];
    if (K.m < m) {
        c->drop_graphs();  // captured graphs hold the old basis pointers
        if (!c->ws_base && K.Q) {
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
            for (auto it = c->owned.begin(); it != c->owned.end(); ++it)
                if (*it == K.Q) { (void)hipFree(K.Q); c->owned.erase(it); break; }
        }
        K.ldq = krylov_ldq((i64)N0, c->layout.ldq_pad);
        K.Q = c->dalloc((size_t)K.ldq * (m + 1) * vec_bytes(basis_prec(p)));
        K.m = m;
    }
    if (!K.z) {
        K.z = gathered_vector(c, (i64)N0, p);
        K.u = c->dalloc(N0 * vec_bytes(basis_prec(p)));
        if (mg16(p)) K.r0 = c->dalloc(N0 * vec_bytes(p));
        K.part = c->dalloc(N0 * vec_bytes(basis_prec(p)));
    }
    ensure_level_vectors(c, p);
    ensure_prec(c, p);
    if (p != P64) ensure_prec(c, P64);
}

size_t plan_bytes(const hpgmx_problem_desc &pd, const hpgmx_mg_desc &mg, int m, unsigned mask, bool cols16,
                  const Layout &lay)
{
    size_t tot = 0;
    auto add = [&](size_t b) { tot += round_up(b ? b : 1); };
    static const size_t vt_bytes[4] = {8, 4, 2, 2};
    bool mat[4] = {true, false, false, false};  // FP64 values always (outer residual)
    bool vt_used[4] = {true, false, false, false};  // FP64 staging always
    for (int p = 0; p < kNumPrec; ++p) {
        if (!((mask >> p) & 1u)) continue;
        mat[matrix_prec((Prec)p)] = true;
        vt_used[vt_of((Prec)p)] = true;
        if (p != P64) vt_used[1] = true;  // FP32 staging (the SpMV output of the 16-bit hierarchy)
    }
    int nx = pd.nx, ny = pd.ny, nz = pd.nz;
    const size_t N0 = (size_t)nx * ny * nz;
    for (int l = 0; l < mg.levels; ++l) {
        const size_t N = (size_t)nx * ny * nz;
        const size_t E = (size_t)ell_entries((i64)N, lay.clog2);
        if (cols16) {
            add(E * sizeof(short));  // 16-bit column offsets and their table
            add(sizeof(ColMap));
        } else {
            add(E * sizeof(int));    // int32 column indices
        }
        for (int q = 0; q < 4; ++q) {
            if (!mat[q]) continue;
            const size_t vb = q == P64 ? 8 : q == P32 ? 4 : 2;
            add(E * vb);
            add(N * vb);
        }
        if (l >= 1)
            for (int vt = 0; vt < 4; ++vt) {
                const bool want = vt == 0 ? (mask & 1u) != 0 : vt == 1 ? (mask & 0xEu) != 0
                                                                       : (mask >> (vt + 2)) & 1u;
                if (want) { add((N + 1) * vt_bytes[vt]); add((N + 1) * vt_bytes[vt]); }
            }
        nx /= 2; ny /= 2; nz /= 2;
    }
    add(sizeof(int));  // the generation's overflow flag
    add(sizeof(Ctrl));
    add((size_t)kMaxRedBlocks * kMaxBasis * 8);
    add(N0 * 8); add((N0 + 1) * 8); add(N0 * 8);  // b, x, r in FP64
    for (int p = 0; p < kNumPrec; ++p) {
        if (!((mask >> p) & 1u)) continue;
        const size_t kb = vec_bytes(basis_prec((Prec)p)), vb = vec_bytes((Prec)p);
        add((size_t)krylov_ldq((i64)N0, lay.ldq_pad) * (m + 1) * kb);
        add((N0 + 1) * vb);
        add(N0 * kb);
        if (mg16((Prec)p)) add(N0 * vb);
        add(N0 * kb);  // partial SpMV sums
    }
    for (int vt = 0; vt < 4; ++vt)  // ABI staging buffers
        if (vt_used[vt]) for (int i = 0; i < 3; ++i) add((N0 + 1) * vt_bytes[vt]);
    return tot;
}

// ---- smoothing and the V-cycle ---------------------------------------------------------------------
// With out.w the sweep's last colour launch also writes the SpMV rows of
// its colour, with out.part the launches at sweep positions 2-6 their
// partial SpMV sums (see SpmvOut).
void sweep_colours(hpgmx_ctx *c, int l, Prec p, const void *r, void *z, bool forward, bool zero,
                   int skip_first_colour, SpmvOut out = {})
{
    const Matrix &A = c->lv[l].A;
    const long long rows = A.g.off[1] - A.g.off[0];
    const bool pairs = zero && !skip_first_colour && gs_pair_possible(A);
    for (int n = 0; n < 8; ++n) {
        const int col = forward ? n : 7 - n;
        if (n == 0 && skip_first_colour) continue;
        // A pair costs colour col ^ 1 two extra evaluations of colour col's
        // rows: cheap when col reads at most 6 slots (the first two pairs of
        // a sweep), 18 or 22 slots for the other two, which pay only on
        // levels 64 times smaller.
        const bool cheap = __builtin_popcount(zero_guess_mask(col, forward)) <= 6;
        if (pairs && rows <= (cheap ? c->layout.pair_rows : c->layout.pair_rows / 64)) {
            ProfScope ps(c, HPGMX_K_GS_ZERO, l);
            launch_gs_pair_zero(A, p, col, forward, r, z, c->stream);
            ++n;
            continue;
        }
        const int mode = !zero ? kGsFull : forward ? kGsZeroForward : kGsZeroBackward;
        ProfScope ps(c, zero ? HPGMX_K_GS_ZERO : HPGMX_K_GS, l);
        SpmvOut o{};
        if (n == 7) { o.w = out.w; o.scale = out.scale; }
        else if (n >= kSplitFirst && out.part) { o.part = out.part; o.forward = forward; }
        launch_gs_colour(A, p, col, mode, r, z, c->stream, o);
    }
}

// `nsweeps` sweeps of kind `kind` on level l; the first starts from z = 0
// when `zero` is set.
void smooth_level(hpgmx_ctx *c, int l, Prec p, int kind, const void *r, void *z, bool zero,
                  int nsweeps, SpmvOut out = {})
{
    if (nsweeps <= 0) {
        if (zero)
            hip_check(hipMemsetAsync(z, 0, (size_t)c->lv[l].A.g.N * vec_bytes(p), c->stream),
                      "hipMemsetAsync");
        return;
    }
    for (int s = 0; s < nsweeps; ++s) {
        const bool zg = zero && s == 0;
        const SpmvOut o = s == nsweeps - 1 ? out : SpmvOut{};
        if (kind == HPGMX_GS_FORWARD) {
            sweep_colours(c, l, p, r, z, true, zg, 0, o);
        } else if (kind == HPGMX_GS_BACKWARD) {
            sweep_colours(c, l, p, r, z, false, zg, 0, o);
        } else {
            sweep_colours(c, l, p, r, z, true, zg, 0);
            // The backward half begins by relaxing colour 7 again with
            // unchanged neighbours, which reproduces its value: skip it.
            sweep_colours(c, l, p, r, z, false, false, 1, o);
        }
    }
}

// The colour whose SpMV rows the V-cycle's last colour launch writes (the
// last colour of the level-0 post-sweep: 7 forward, 0 backward and
// symmetric), or -1 when the V-cycle does not end with a full sweep on level
// 0 (one level, or no post-sweep).
int fused_spmv_colour(const hpgmx_ctx *c)
{
    if (c->mg.levels < 2 || c->mg.post_sweeps < 1) return -1;
    return c->mg.sweep == HPGMX_GS_FORWARD ? 7 : 0;
}

// A pre-smoother of one forward or backward sweep from z = 0 lets the fused
// restriction use the shortcut of k_restrict_after_sweep.
bool restrict_after_single_sweep(int kind, int nsweeps)
{
    return nsweeps == 1 && (kind == HPGMX_GS_FORWARD || kind == HPGMX_GS_BACKWARD);
}

// The first half of a V-cycle level: z <- nsweeps sweeps of kind `kind` from
// z = 0 on level l, then rc = R (r - A z) on level l + 1 (eq. (6)).
void presmooth_restrict(hpgmx_ctx *c, int l, Prec p, int kind, int nsweeps, const void *r, void *z, void *rc)
{
    smooth_level(c, l, p, kind, r, z, true, nsweeps);
    ProfScope ps(c, HPGMX_K_RESTRICT, l);
    const Geom &gc = c->lv[l + 1].A.g;
    if (restrict_after_single_sweep(kind, nsweeps))
        launch_restrict_after_sweep(c->lv[l].A, gc, p, kind == HPGMX_GS_FORWARD, z, rc, c->stream);
    else
        launch_restrict(c->lv[l].A, gc, p, r, z, rc, c->stream);
}

// z = M^{-1} r on level l (z is overwritten; the cycle starts from zero).
// With out.w (level 0 only, see fused_spmv_colour) the last colour launch
// also writes its rows of w = A z.
void vcycle(hpgmx_ctx *c, int l, Prec p, const void *r, void *z, SpmvOut out = {})
{
    const hpgmx_mg_desc &mg = c->mg;
    const int vt = vt_of(p);
    if (l == mg.levels - 1) {
        smooth_level(c, l, p, mg.sweep, r, z, true, mg.coarsest_sweeps);
        return;
    }
    Level &C = c->lv[l + 1];
    presmooth_restrict(c, l, p, mg.sweep, mg.pre_sweeps, r, z, C.r[vt]);
    vcycle(c, l + 1, p, C.r[vt], C.z[vt]);
    {
        ProfScope ps(c, HPGMX_K_PROLONG, l);
        launch_prolong(c->lv[l].A.g, C.A.g, p, C.z[vt], z, c->stream);
    }
    smooth_level(c, l, p, mg.sweep, r, z, false, mg.post_sweeps, out);
}

// ---- GMRES-IR (Alg. 3) ----------------------------------------------------------------------------------
struct Scal {  // mirrors the scalar block of Ctrl
    double rho, inv_rho, beta, inv_beta, nrm2, rho0;
    int breakdown, nonfinite;
};

Scal read_scal(hpgmx_ctx *c)
{
    hip_check(hipMemcpyAsync(c->host_scal, &c->ctrl->rho, sizeof(Scal), hipMemcpyDeviceToHost,
                             c->stream), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    Scal s;
    std::memcpy(&s, c->host_scal, sizeof(Scal));
    return s;
}

// Inner steps are pipelined one deep: the host enqueues step k + 1 before it
// waits for the scalars of step k, so the GPU does not idle for the host's
// round trip.  The copy of step k's scalars goes to slot k & 1 of the
// pinned buffer and the host waits on that slot's event only.  A step
// enqueued past the end of a cycle (convergence, breakdown) is discarded: it
// writes only Hessenberg column k + 1, t from index k + 1 on and basis
// column k + 2, which the back-solve and the basis combination of a cycle
// of k + 1 steps never read, and the next cycle starts afresh.  No step is
// enqueued past the restart length or the iteration limit.
void ensure_scal_events(hpgmx_ctx *c)
{
    for (auto &e : c->ev_scal)
        if (!e) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
}

void enqueue_scal(hpgmx_ctx *c, const Ctrl *ctrl, int K, double *host, int slot)
{
    char *dst = (char *)host + (size_t)slot * K * 64;
    if (K == 1)
        hip_check(hipMemcpyAsync(dst, &ctrl->rho, sizeof(Scal), hipMemcpyDeviceToHost, c->stream),
                  "hipMemcpyAsync");
    else
        hip_check(hipMemcpy2DAsync(dst, sizeof(Scal), &ctrl[0].rho, sizeof(Ctrl), sizeof(Scal), K,
                                   hipMemcpyDeviceToHost, c->stream),
                  "hipMemcpy2DAsync");
    hip_check(hipEventRecord(c->ev_scal[slot], c->stream), "hipEventRecord");
}

void wait_scal(hpgmx_ctx *c, int K, const double *host, int slot, Scal *out)
{
    hip_check(hipEventSynchronize(c->ev_scal[slot]), "hipEventSynchronize");
    std::memcpy(out, (const char *)host + (size_t)slot * K * 64, K * sizeof(Scal));
}

// Graph replay needs a capturable stream and no memset nodes (a level with
// zero sweeps clears its vector with a memset); profiling times single
// launches, so it runs eagerly.
bool graphs_allowed(const hpgmx_ctx *c, const hpgmx_solve_desc *d)
{
    const hpgmx_mg_desc &mgd = c->mg;
    return (d->flags & HPGMX_SOLVE_GRAPH) && !c->prof && mgd.pre_sweeps > 0 && mgd.post_sweeps > 0 &&
           mgd.coarsest_sweeps > 0;
}

// While alive (and `on`), the handle's work goes to its private stream,
// ordered after the work already on the caller's stream and before the
// caller's later work.
struct GraphStream {
    hpgmx_ctx *c;
    hipStream_t user;
    bool on;
    GraphStream(hpgmx_ctx *c_, bool on_) : c(c_), user(c_->stream), on(on_)
    {
        if (!on) return;
        if (!c->own) {
            hip_check(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking), "hipStreamCreateWithFlags");
            hip_check(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming), "hipEventCreate");
            hip_check(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming), "hipEventCreate");
        }
        hip_check(hipEventRecord(c->ev_in, user), "hipEventRecord");
        hip_check(hipStreamWaitEvent(c->own, c->ev_in, 0), "hipStreamWaitEvent");
        c->stream = c->own;
    }
    ~GraphStream()
    {
        if (!on) return;
        (void)hipEventRecord(c->ev_out, c->stream);
        (void)hipStreamWaitEvent(user, c->ev_out, 0);
        c->stream = user;
    }
};

// Runs `step` as an instantiated graph: captured on first use of `key`,
// replayed afterwards.
template <typename F>
void replay_step(hpgmx_ctx *c, const std::tuple<int, int, int, int> &key, F &&step)
{
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        hip_check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        step();
        hip_check(hipStreamEndCapture(c->stream, &g), "hipStreamEndCapture");
        hip_check(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "hipGraphInstantiate");
        (void)hipGraphDestroy(g);
        it = c->graphs.emplace(key, ge).first;
    }
    hip_check(hipGraphLaunch(it->second, c->stream), "hipGraphLaunch");
}

hpgmx_status solve(hpgmx_ctx *c, const double *b, double *x, const hpgmx_solve_desc *d,
                   hpgmx_solve_stats *st)
{
    const int m = d->restart;
    const Prec p = (Prec)d->inner_dtype;
    ensure_krylov(c, p, m);
    Krylov &K = c->kry[p];
    const Matrix &A0 = c->lv[0].A;
    const Geom &g0 = A0.g;
    const i64 N = g0.N;
    const Prec bp = basis_prec(p);  // Krylov vectors: FP64 or FP32
    const bool mg = mg16(p);        // 16-bit multigrid hierarchy
    const size_t vb = vec_bytes(bp);
    char *Q = (char *)K.Q;
    const i64 ldq = K.ldq;
    auto col = [&](int j) { return (void *)(Q + (size_t)j * ldq * vb); };

    c->prof = (d->flags & HPGMX_SOLVE_PROFILE) != 0;
    // Graph replay needs a capturable stream and no memset nodes (a level with
    // zero sweeps clears its vector with a memset); profiling times single
    // launches, so it runs eagerly.
    const bool use_graph = graphs_allowed(c, d);
    GraphStream gs_scope(c, use_graph);
    if (c->prof) {
        std::memset(c->prof_ms, 0, sizeof(c->prof_ms));
        std::memset(c->prof_n, 0, sizeof(c->prof_n));
        c->evused = 0;
    }
    hpgmx_solve_stats S{};
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    hip_check(hipEventRecord(e0, c->stream), "hipEventRecord");

    {
        ProfScope ps(c, HPGMX_K_PERMUTE, 0);
        launch_nat2int(g0, P64, b, P64, c->b_int, c->stream);
    }
    {
        ProfScope ps(c, HPGMX_K_PERMUTE, 0);
        launch_nat2int(g0, P64, x, P64, c->x_int, c->stream);
    }
    launch_norm64(N, 1, c->b_int, c->partials, c->ctrl, kFinishRho0, 0, c->stream);
    Scal sc = read_scal(c);
    const double rho0 = sc.rho0;
    S.rho0 = rho0;
    hpgmx_status status = HPGMX_OK;
    if (sc.nonfinite) {
        status = HPGMX_ENONFINITE;
        c->err = "right-hand side is not finite";
    } else if (rho0 == 0.0) {
        hip_check(hipMemsetAsync(x, 0, (size_t)N * 8, c->stream), "hipMemsetAsync");
        S.converged = 1;
        S.final_rel_res = 0.0;
    } else {
        int its = 0;
        for (;;) {
            {
                PassScope ps(c, HPGMX_K_RESID64, 0);
                launch_resid64(A0, c->x_int, c->b_int, c->r64, c->partials, c->ctrl, m, c->stream);
            }
            sc = read_scal(c);
            double rho = sc.rho;
            S.final_rel_res = rho / rho0;
            if (sc.nonfinite) { status = HPGMX_ENONFINITE; c->err = "outer residual is not finite"; break; }
            if (rho / rho0 < d->tol) { S.converged = 1; break; }
            if (its >= d->max_iters) break;
            {
                ProfScope ps(c, HPGMX_K_CAST, 0);
                launch_cast(N, 1, bp, c->r64, c->ctrl, col(0), c->stream);
            }
            int kk = 0;
            ensure_scal_events(c);
            // one inner step: z = M^{-1} q_k, w = A z, CGS2, Givens, q_{k+1},
            // then the copy of its scalars (see enqueue_scal)
            auto run_step = [&](int k) {
                auto step = [&]() {
                    // w = A z: with kSpmvLast the rows of colour fc come from
                    // the V-cycle's last colour launch, the others from the
                    // SpMV; with kSpmvSplit the launches at sweep positions
                    // 2-6 also leave partial sums for their rows
                    const int fc = fused_spmv_colour(c);
                    const int sm = fc < 0 ? kSpmvPlain : c->spmv_mode;
                    SpmvOut out{};
                    if (sm == kSpmvLast || sm == kSpmvSplit) { out.w = col(k + 1); out.scale = spmv_scale(p, c->ctrl, k); }
                    if (sm == kSpmvSplit) out.part = K.part;
                    if (mg) {
                        {
                            ProfScope ps(c, HPGMX_K_CAST, 0);
                            launch_cast_mg(N, p, (const float *)col(k), c->ctrl, false, k, K.r0, c->stream);
                        }
                        vcycle(c, 0, p, K.r0, K.z, out);
                    } else {
                        vcycle(c, 0, p, col(k), K.z, out);
                    }
                    {
                        ProfScope ps(c, HPGMX_K_SPMV, 0);
                        if (sm == kSpmvSplit || sm == kSpmvSplitSeparate)
                            launch_spmv_split(A0, p, K.z, col(k + 1), K.part, fc == 7, sm == kSpmvSplit, c->stream,
                                              c->ctrl, k);
                        else
                            launch_spmv(A0, p, K.z, col(k + 1), c->stream, c->ctrl, k, sm == kSpmvLast ? fc : -1);
                    }
                    {
                        PassScope ps(c, HPGMX_K_DOT, 0);
                        launch_dot(N, 1, bp, K.Q, ldq, k + 1, col(k + 1), c->partials, c->ctrl, c->stream);
                    }
                    {
                        PassScope ps(c, HPGMX_K_CGS_DOT, 0);
                        launch_cgs_dot(N, 1, bp, K.Q, ldq, k + 1, col(k + 1), c->partials, c->ctrl, c->stream);
                    }
                    {
                        PassScope ps(c, HPGMX_K_CGS_NORM, 0);
                        launch_cgs_norm(N, 1, bp, K.Q, ldq, k + 1, col(k + 1), c->partials, c->ctrl, k, m, c->stream);
                    }
                };
                if (use_graph) replay_step(c, std::make_tuple((int)p, k, m, 1), step);
                else step();
                enqueue_scal(c, c->ctrl, 1, c->host_scal, k & 1);
            };
            if (!(rho / rho0 < d->tol)) {
                run_step(0);
                for (int k = 0; k < m; ++k) {
                    const bool next = k + 1 < m && its + 1 < d->max_iters;
                    if (next) run_step(k + 1);  // ahead of the test on step k
                    wait_scal(c, 1, c->host_scal, k & 1, &sc);
                    rho = sc.rho;
                    kk = k + 1;
                    ++its;
                    if (d->res_hist_host && its - 1 < d->res_hist_len) d->res_hist_host[its - 1] = rho / rho0;
                    S.est_rel_res = rho / rho0;
                    if (sc.nonfinite) break;
                    if (sc.breakdown) { S.breakdown = 1; break; }
                    if (its >= d->max_iters) break;
                    if (rho / rho0 < d->tol) break;
                    if (!next) break;
                }
            }
            if (sc.nonfinite) { status = HPGMX_ENONFINITE; c->err = "Krylov vector is not finite"; break; }
            {
                ProfScope ps(c, HPGMX_K_TRSM, 0);
                launch_trsm(c->ctrl, KCount{{kk}}, 1, m, c->stream);
            }
            c->last_k[p] = kk;
            c->last_m[p] = m;
            {
                ProfScope ps(c, HPGMX_K_GEMV, 0);
                launch_gemv(N, 1, bp, K.Q, ldq, kk, c->ctrl, K.u, c->stream);
            }
            if (mg) {
                {
                    ProfScope ps(c, HPGMX_K_CAST, 0);
                    launch_cast_mg(N, p, (const float *)K.u, c->ctrl, true, kk, K.r0, c->stream);
                }
                vcycle(c, 0, p, K.r0, K.z);
            } else {
                vcycle(c, 0, p, K.u, K.z);
            }
            {
                ProfScope ps(c, HPGMX_K_UPDATE, 0);
                launch_update(N, p, K.z, c->x_int, c->stream, c->ctrl);
            }
            ++S.restarts;
        }
        S.iters = its;
        {
            ProfScope ps(c, HPGMX_K_PERMUTE, 0);
            launch_int2nat(g0, P64, c->x_int, P64, x, c->stream);
        }
    }
    hip_check(hipEventRecord(e1, c->stream), "hipEventRecord");
    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    S.solve_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (c->prof) c->prof_collect();
    c->prof = false;
    if (st) *st = S;
    return status;
}

// ---- batched solves ------------------------------------------------------------------------------
int batch_width(int nrhs) { return nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : 8; }

void *gathered_batch(hpgmx_ctx *c, i64 N, int K, Prec p)
{
    const size_t vb = vec_bytes(p);
    char *v = (char *)c->dalloc((size_t)(N + 1) * K * vb);
    hip_check(hipMemsetAsync(v + (size_t)N * K * vb, 0, K * vb, c->stream), "hipMemsetAsync");
    return v;
}

// The staging buffers serve every level: re-zero row N of the level used.
void zero_batch_row(hpgmx_ctx *c, void *v, i64 N, int K, Prec p)
{
    const size_t vb = vec_bytes(p);
    hip_check(hipMemsetAsync((char *)v + (size_t)N * K * vb, 0, K * vb, c->stream), "hipMemsetAsync");
}

Batch &ensure_batch(hpgmx_ctx *c, int K)
{
    Batch &B = c->batches[K];
    if (B.K) return B;
    const i64 N0 = c->lv[0].A.g.N;
    B.b = (double *)c->dalloc((size_t)N0 * K * 8);
    B.x = (double *)gathered_batch(c, N0, K, P64);
    B.r64 = (double *)c->dalloc((size_t)N0 * K * 8);
    B.ctrl = (Ctrl *)c->dalloc(K * sizeof(Ctrl));
    hip_check(hipMemsetAsync(B.ctrl, 0, K * sizeof(Ctrl), c->stream), "hipMemsetAsync");
    B.partials = (double *)c->dalloc((size_t)kMaxRedBlocks * kMaxBasis * K * 8);
    if (!B.host_scal)
        hip_check(hipHostMalloc((void **)&B.host_scal, (size_t)2 * K * 64, hipHostMallocDefault), "hipHostMalloc");
    B.K = K;
    return B;
}

// Level vectors and (m > 0) the Krylov workspace of vector type p.
void ensure_batch_prec(hpgmx_ctx *c, Batch &B, Prec p, int m)
{
    const int vt = vt_of(p), K = B.K;
    ensure_prec(c, p);
    ensure_prec(c, P64);
    for (size_t l = 1; l < c->lv.size(); ++l) {
        if (!B.lr[vt][l]) {
            B.lr[vt][l] = gathered_batch(c, c->lv[l].A.g.N, K, p);
            B.lz[vt][l] = gathered_batch(c, c->lv[l].A.g.N, K, p);
        }
    }
    if (m <= 0) return;
    const i64 N0 = c->lv[0].A.g.N;
    Krylov &Kr = B.kry[vt];
    if (Kr.m < m) {
        c->drop_graphs();
        if (!c->ws_base && Kr.Q) {
            hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
            for (auto it = c->owned.begin(); it != c->owned.end(); ++it)
                if (*it == Kr.Q) { (void)hipFree(Kr.Q); c->owned.erase(it); break; }
        }
        Kr.ldq = krylov_ldq(N0 * K, c->layout.ldq_pad);
        Kr.Q = c->dalloc((size_t)Kr.ldq * (m + 1) * vec_bytes(p));
        Kr.m = m;
    }
    if (!Kr.z) {
        Kr.z = gathered_batch(c, N0, K, p);
        Kr.u = c->dalloc((size_t)N0 * K * vec_bytes(p));
        Kr.part = c->dalloc((size_t)N0 * K * vec_bytes(p));
    }
}

void ensure_batch_tmp(hpgmx_ctx *c, Batch &B, int vt)
{
    const i64 N0 = c->lv[0].A.g.N;
    for (int i = 0; i < 3; ++i)
        if (!B.tmp[vt][i]) B.tmp[vt][i] = gathered_batch(c, N0, B.K, vt == 0 ? P64 : P32);
}

// R of a batched kernel: the adopted table, else the fixed rule (every lane
// takes the whole row on large levels, one right-hand side per lane on
// small ones, where parallelism is scarce).
int tile_r(const hpgmx_ctx *c, const Batch &B, Prec p, int kind, int l)
{
    const int R = B.tune[p].R[kind][l];
    if (R > 0) return R;
    return c->lv[l].A.g.N * B.K >= (1ll << 22) ? B.K : 1;
}

// With out.y / out.part as sweep_colours() with SpmvOut.
void bsweep_colours(hpgmx_ctx *c, Batch &B, int l, Prec p, const void *r, void *z, bool forward, bool zero,
                    int skip_first_colour, BSpmvOut out = {})
{
    const Matrix &A = c->lv[l].A;
    const int R = tile_r(c, B, p, zero ? HPGMX_BK_GS_ZERO : HPGMX_BK_GS, l);
    for (int n = 0; n < 8; ++n) {
        const int col = forward ? n : 7 - n;
        if (n == 0 && skip_first_colour) continue;
        const int mode = !zero ? kGsFull : forward ? kGsZeroForward : kGsZeroBackward;
        ProfScope ps(c, zero ? HPGMX_K_GS_ZERO : HPGMX_K_GS, l);
        BSpmvOut o{};
        if (n == 7) { o.y = out.y; o.ctrl = out.ctrl; o.k = out.k; }
        else if (n >= kSplitFirst && out.part) { o.part = out.part; o.forward = forward; }
        launch_bgs_colour(A, p, B.K, R, col, mode, r, z, c->stream, o);
    }
}

void bsmooth_level(hpgmx_ctx *c, Batch &B, int l, Prec p, int kind, const void *r, void *z, bool zero,
                   int nsweeps, BSpmvOut out = {})
{
    if (nsweeps <= 0) {
        if (zero)
            hip_check(hipMemsetAsync(z, 0, (size_t)c->lv[l].A.g.N * B.K * vec_bytes(p), c->stream),
                      "hipMemsetAsync");
        return;
    }
    for (int s = 0; s < nsweeps; ++s) {
        const bool zg = zero && s == 0;
        const BSpmvOut o = s == nsweeps - 1 ? out : BSpmvOut{};
        if (kind == HPGMX_GS_FORWARD) {
            bsweep_colours(c, B, l, p, r, z, true, zg, 0, o);
        } else if (kind == HPGMX_GS_BACKWARD) {
            bsweep_colours(c, B, l, p, r, z, false, zg, 0, o);
        } else {
            bsweep_colours(c, B, l, p, r, z, true, zg, 0);
            bsweep_colours(c, B, l, p, r, z, false, false, 1, o);  // colour 7 is unchanged
        }
    }
}

// presmooth_restrict() for K right-hand sides at once.
void bpresmooth_restrict(hpgmx_ctx *c, Batch &B, int l, Prec p, int kind, int nsweeps, const void *r, void *z,
                         void *rc)
{
    bsmooth_level(c, B, l, p, kind, r, z, true, nsweeps);
    ProfScope ps(c, HPGMX_K_RESTRICT, l);
    const Geom &gc = c->lv[l + 1].A.g;
    const int R = tile_r(c, B, p, HPGMX_BK_RESTRICT, l);
    if (restrict_after_single_sweep(kind, nsweeps))
        launch_brestrict_after_sweep(c->lv[l].A, gc, p, B.K, R, kind == HPGMX_GS_FORWARD, z, rc, c->stream);
    else
        launch_brestrict(c->lv[l].A, gc, p, B.K, R, r, z, rc, c->stream);
}

// The V-cycle of vcycle() for K right-hand sides at once (out: as vcycle()).
void bvcycle(hpgmx_ctx *c, Batch &B, int l, Prec p, const void *r, void *z, BSpmvOut out = {})
{
    const hpgmx_mg_desc &mg = c->mg;
    const int vt = vt_of(p);
    if (l == mg.levels - 1) {
        bsmooth_level(c, B, l, p, mg.sweep, r, z, true, mg.coarsest_sweeps);
        return;
    }
    const Geom &gc = c->lv[l + 1].A.g;
    bpresmooth_restrict(c, B, l, p, mg.sweep, mg.pre_sweeps, r, z, B.lr[vt][l + 1]);
    bvcycle(c, B, l + 1, p, B.lr[vt][l + 1], B.lz[vt][l + 1]);
    {
        ProfScope ps(c, HPGMX_K_PROLONG, l);
        launch_bprolong(c->lv[l].A.g, gc, p, B.K, B.lz[vt][l + 1], z, c->stream);
    }
    bsmooth_level(c, B, l, p, mg.sweep, r, z, false, mg.post_sweeps, out);
}

// Times every R for every batched kernel kind and level (on zeroed staging
// vectors) and adopts the fastest.
void autotune(hpgmx_ctx *c, Batch &B, Prec p)
{
    const int vt = vt_of(p), K = B.K;
    ensure_batch_prec(c, B, p, 0);
    ensure_batch_tmp(c, B, vt);
    ensure_batch_tmp(c, B, 0);
    const i64 N0 = c->lv[0].A.g.N;
    for (int w = 0; w < 2; ++w)
        for (int i = 0; i < 3; ++i)
            if (B.tmp[w][i])
                hip_check(hipMemsetAsync(B.tmp[w][i], 0, (size_t)(N0 + 1) * K * (w == 0 ? 8 : 4), c->stream),
                          "hipMemsetAsync");
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    constexpr int kReps = 5;
    auto time_it = [&](auto &&launch) -> double {
        launch();
        hip_check(hipEventRecord(e0, c->stream), "hipEventRecord");
        for (int r = 0; r < kReps; ++r) launch();
        hip_check(hipEventRecord(e1, c->stream), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        return ms / kReps;
    };
    BatchTune T{};
    for (int k = 0; k < HPGMX_BK_COUNT; ++k)
        for (int l = 0; l < kMaxLevels; ++l) T.ms[k][l] = -1.0;
    void *t0 = B.tmp[vt][0], *t1 = B.tmp[vt][1], *t2 = B.tmp[vt][2];
    const int L = (int)c->lv.size();
    for (int l = 0; l < L; ++l) {
        const Matrix &A = c->lv[l].A;
        for (int R = 1; R <= K; R *= 2) {
            double t[HPGMX_BK_COUNT];
            for (double &v : t) v = -1.0;
            t[HPGMX_BK_SPMV] = time_it([&] { launch_bspmv(A, p, K, R, t0, t1, c->stream); });
            t[HPGMX_BK_GS] = time_it([&] {
                for (int col = 0; col < 8; ++col) launch_bgs_colour(A, p, K, R, col, kGsFull, t0, t1, c->stream);
            });
            t[HPGMX_BK_GS_ZERO] = time_it([&] {
                for (int col = 0; col < 8; ++col)
                    launch_bgs_colour(A, p, K, R, col, kGsZeroForward, t0, t1, c->stream);
            });
            if (l + 1 < L)
                t[HPGMX_BK_RESTRICT] = time_it([&] {  // the variant the V-cycle uses
                    if (restrict_after_single_sweep(c->mg.sweep, c->mg.pre_sweeps))
                        launch_brestrict_after_sweep(A, c->lv[l + 1].A.g, p, K, R, c->mg.sweep == HPGMX_GS_FORWARD,
                                                     t1, t2, c->stream);
                    else
                        launch_brestrict(A, c->lv[l + 1].A.g, p, K, R, t0, t1, t2, c->stream);
                });
            if (l == 0)
                t[HPGMX_BK_RESID64] = time_it([&] {
                    launch_bresid64(A, K, R, (const double *)B.tmp[0][0], (const double *)B.tmp[0][1],
                                    (double *)B.tmp[0][2], B.partials, B.ctrl, 1, c->stream);
                });
            for (int k = 0; k < HPGMX_BK_COUNT; ++k) {
                if (t[k] < 0.0) continue;
                if (T.ms[k][l] < 0.0 || t[k] < T.ms[k][l]) {
                    T.ms[k][l] = t[k];
                    T.R[k][l] = R;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int k = 0; k < HPGMX_BK_COUNT; ++k)
        for (int l = 0; l < kMaxLevels; ++l)
            if (T.ms[k][l] < 0.0) T.ms[k][l] = 0.0;
    T.set = true;
    B.tune[p] = T;
    c->drop_graphs();  // captured steps hold the old tiles
}

void read_scal_batch(hpgmx_ctx *c, Batch &B, Scal *out)
{
    hip_check(hipMemcpy2DAsync(B.host_scal, sizeof(Scal), &B.ctrl[0].rho, sizeof(Ctrl), sizeof(Scal), B.K,
                               hipMemcpyDeviceToHost, c->stream),
              "hipMemcpy2DAsync");
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    std::memcpy(out, B.host_scal, B.K * sizeof(Scal));
}

hpgmx_status bsolve(hpgmx_ctx *c, int nrhs, const double *Bn, double *Xn, const hpgmx_solve_desc *d,
                    hpgmx_solve_stats *st)
{
    const int m = d->restart;
    const Prec p = (Prec)d->inner_dtype;
    const int K = batch_width(nrhs);
    Batch &B = ensure_batch(c, K);
    ensure_batch_prec(c, B, p, m);
    if ((d->flags & HPGMX_SOLVE_AUTOTUNE) && !B.tune[p].set) autotune(c, B, p);
    Krylov &Kr = B.kry[vt_of(p)];
    const Matrix &A0 = c->lv[0].A;
    const Geom &g0 = A0.g;
    const i64 N = g0.N, M = N * K;
    const size_t vb = vec_bytes(p);
    char *Q = (char *)Kr.Q;
    const i64 ldq = Kr.ldq;
    auto col = [&](int j) { return (void *)(Q + (size_t)j * ldq * vb); };

    c->prof = (d->flags & HPGMX_SOLVE_PROFILE) != 0;
    const bool use_graph = graphs_allowed(c, d);
    GraphStream gs_scope(c, use_graph);
    if (c->prof) {
        std::memset(c->prof_ms, 0, sizeof(c->prof_ms));
        std::memset(c->prof_n, 0, sizeof(c->prof_n));
        c->evused = 0;
    }
    hpgmx_solve_stats S[kMaxBatch] = {};
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    hip_check(hipEventRecord(e0, c->stream), "hipEventRecord");
    {
        ProfScope ps(c, HPGMX_K_PERMUTE, 0);
        launch_bnat2int(g0, P64, P64, K, nrhs, Bn, B.b, c->stream);
    }
    {
        ProfScope ps(c, HPGMX_K_PERMUTE, 0);
        launch_bnat2int(g0, P64, P64, K, nrhs, Xn, B.x, c->stream);
    }
    launch_norm64(M, K, B.b, B.partials, B.ctrl, kFinishRho0, 0, c->stream);
    Scal sc[kMaxBatch];
    read_scal_batch(c, B, sc);
    double rho0[kMaxBatch], rho[kMaxBatch];
    bool done[kMaxBatch];
    int its[kMaxBatch] = {};
    hpgmx_status status = HPGMX_OK;
    for (int j = 0; j < K; ++j) {
        rho0[j] = sc[j].rho0;
        S[j].rho0 = rho0[j];
        if (j < nrhs && sc[j].nonfinite) {
            status = HPGMX_ENONFINITE;
            c->err = "right-hand side " + std::to_string(j) + " is not finite";
        }
        done[j] = rho0[j] == 0.0;  // b = 0: x = 0 (set below)
        if (done[j]) S[j].converged = 1;
    }
    if (status == HPGMX_OK) {
        for (;;) {
            {
                PassScope ps(c, HPGMX_K_RESID64, 0);
                launch_bresid64(A0, K, tile_r(c, B, p, HPGMX_BK_RESID64, 0), B.x, B.b, B.r64, B.partials, B.ctrl,
                                m, c->stream);
            }
            read_scal_batch(c, B, sc);
            bool bad = false, any = false;
            for (int j = 0; j < K; ++j) {
                rho[j] = sc[j].rho;
                if (done[j]) continue;
                S[j].final_rel_res = rho[j] / rho0[j];
                if (sc[j].nonfinite) { bad = true; continue; }
                if (rho[j] / rho0[j] < d->tol) { S[j].converged = 1; done[j] = true; continue; }
                if (its[j] >= d->max_iters) { done[j] = true; continue; }
                any = true;
            }
            if (bad) { status = HPGMX_ENONFINITE; c->err = "outer residual is not finite"; break; }
            if (!any) break;
            {
                ProfScope ps(c, HPGMX_K_CAST, 0);
                launch_cast(M, K, p, B.r64, B.ctrl, col(0), c->stream);
            }
            int kk[kMaxBatch] = {};
            bool cyc[kMaxBatch];
            for (int j = 0; j < K; ++j) cyc[j] = !done[j];
            bool nonfin = false;
            ensure_scal_events(c);
            // one inner step for every right-hand side: z = M^{-1} q_k, w = A z,
            // CGS2, Givens, q_{k+1}, then the copy of the scalars (pipelined one
            // deep as in solve(); see enqueue_scal)
            auto run_step = [&](int k) {
                auto step = [&]() {
                    // w = A z shared with the V-cycle's last sweep as in solve()
                    // (FP32 and FP64 batches; the last colour alone is not
                    // offered: kSpmvLast runs as kSpmvPlain)
                    const int fc = fused_spmv_colour(c);
                    const int sm = fc < 0 || (p != P32 && p != P64) || c->spmv_mode == kSpmvLast ? kSpmvPlain
                                                                                                  : c->spmv_mode;
                    BSpmvOut out{};
                    if (sm == kSpmvSplit) { out.y = col(k + 1); out.ctrl = B.ctrl; out.k = k; out.part = Kr.part; }
                    bvcycle(c, B, 0, p, col(k), Kr.z, out);
                    {
                        ProfScope ps(c, HPGMX_K_SPMV, 0);
                        const int Rs = tile_r(c, B, p, HPGMX_BK_SPMV, 0);
                        if (sm == kSpmvSplit || sm == kSpmvSplitSeparate)
                            launch_bspmv_split(A0, p, K, Rs, Kr.z, col(k + 1), Kr.part, fc == 7, sm == kSpmvSplit,
                                               c->stream, B.ctrl, k);
                        else
                            launch_bspmv(A0, p, K, Rs, Kr.z, col(k + 1), c->stream, B.ctrl, k);
                    }
                    {
                        PassScope ps(c, HPGMX_K_DOT, 0);
                        launch_dot(M, K, p, Kr.Q, ldq, k + 1, col(k + 1), B.partials, B.ctrl, c->stream);
                    }
                    {
                        PassScope ps(c, HPGMX_K_CGS_DOT, 0);
                        launch_cgs_dot(M, K, p, Kr.Q, ldq, k + 1, col(k + 1), B.partials, B.ctrl, c->stream);
                    }
                    {
                        PassScope ps(c, HPGMX_K_CGS_NORM, 0);
                        launch_cgs_norm(M, K, p, Kr.Q, ldq, k + 1, col(k + 1), B.partials, B.ctrl, k, m, c->stream);
                    }
                };
                if (use_graph) replay_step(c, std::make_tuple((int)p, k, m, K), step);
                else step();
                enqueue_scal(c, B.ctrl, K, B.host_scal, k & 1);
            };
            // right-hand sides still taking steps in this cycle (the test at
            // the top of Alg. 3's inner loop)
            auto any_active = [&]() {
                bool act = false;
                for (int j = 0; j < K; ++j) {
                    if (cyc[j] && rho[j] / rho0[j] < d->tol) cyc[j] = false;
                    act = act || cyc[j];
                }
                return act;
            };
            if (any_active()) {
                run_step(0);
                for (int k = 0; k < m; ++k) {
                    bool more = false;  // some right-hand side may take step k + 1
                    for (int j = 0; j < K; ++j) more = more || (cyc[j] && its[j] + 1 < d->max_iters);
                    const bool next = k + 1 < m && more;
                    if (next) run_step(k + 1);  // ahead of the tests on step k
                    wait_scal(c, K, B.host_scal, k & 1, sc);
                    for (int j = 0; j < K; ++j) {
                        if (!cyc[j]) continue;
                        rho[j] = sc[j].rho;
                        kk[j] = k + 1;
                        ++its[j];
                        if (d->res_hist_host && j < nrhs && its[j] - 1 < d->res_hist_len)
                            d->res_hist_host[(size_t)j * d->res_hist_len + its[j] - 1] = rho[j] / rho0[j];
                        S[j].est_rel_res = rho[j] / rho0[j];
                        if (sc[j].nonfinite) { nonfin = true; cyc[j] = false; continue; }
                        if (sc[j].breakdown) { S[j].breakdown = 1; cyc[j] = false; continue; }
                        if (its[j] >= d->max_iters) cyc[j] = false;
                    }
                    if (nonfin) break;
                    if (!any_active() || !next) break;
                }
            }
            if (nonfin) { status = HPGMX_ENONFINITE; c->err = "Krylov vector is not finite"; break; }
            KCount kc{};
            int kmax = 0;
            for (int j = 0; j < K; ++j) {
                kc.v[j] = kk[j];
                kmax = kk[j] > kmax ? kk[j] : kmax;
                if (kk[j] > 0) ++S[j].restarts;
            }
            {
                ProfScope ps(c, HPGMX_K_TRSM, 0);
                launch_trsm(B.ctrl, kc, K, m, c->stream);
            }
            {
                ProfScope ps(c, HPGMX_K_GEMV, 0);
                launch_gemv(M, K, p, Kr.Q, ldq, kmax, B.ctrl, Kr.u, c->stream);
            }
            bvcycle(c, B, 0, p, Kr.u, Kr.z);
            {
                ProfScope ps(c, HPGMX_K_UPDATE, 0);
                launch_update(M, p, Kr.z, B.x, c->stream);
            }
        }
        for (int j = 0; j < K; ++j) S[j].iters = its[j];
        {
            ProfScope ps(c, HPGMX_K_PERMUTE, 0);
            launch_bint2nat(g0, P64, P64, K, nrhs, B.x, Xn, c->stream);
        }
        for (int j = 0; j < nrhs; ++j)
            if (rho0[j] == 0.0)
                hip_check(hipMemsetAsync(Xn + (size_t)j * N, 0, (size_t)N * 8, c->stream), "hipMemsetAsync");
    }
    hip_check(hipEventRecord(e1, c->stream), "hipEventRecord");
    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (c->prof) c->prof_collect();
    c->prof = false;
    if (st)
        for (int j = 0; j < nrhs; ++j) {
            st[j] = S[j];
            st[j].solve_ms = ms;
        }
    return status;
}

size_t plan_batch_bytes(const hpgmx_problem_desc &pd, const hpgmx_mg_desc &mg, int nrhs, int m, unsigned mask,
                        const Layout &lay)
{
    const int K = batch_width(nrhs);
    size_t tot = 0;
    auto add = [&](size_t b) { tot += round_up(b ? b : 1); };
    const size_t N0 = (size_t)pd.nx * pd.ny * pd.nz;
    add(N0 * K * 8); add((N0 + 1) * K * 8); add(N0 * K * 8);  // b, x, r in FP64
    add(K * sizeof(Ctrl));
    add((size_t)kMaxRedBlocks * kMaxBasis * K * 8);
    for (int vt = 0; vt < 2; ++vt) {
        const bool want = vt == 0 ? (mask & 1u) != 0 : (mask & 0xEu) != 0;  // FP32 vectors for F32/F16/BF16
        if (!want) continue;
        const size_t vb = vt == 0 ? 8 : 4;
        int nx = pd.nx / 2, ny = pd.ny / 2, nz = pd.nz / 2;
        for (int l = 1; l < mg.levels; ++l) {
            const size_t N = (size_t)nx * ny * nz;
            add((N + 1) * K * vb);
            add((N + 1) * K * vb);
            nx /= 2; ny /= 2; nz /= 2;
        }
        add((size_t)krylov_ldq((i64)(N0 * K), lay.ldq_pad) * (m + 1) * vb);
        add((N0 + 1) * K * vb);
        add(N0 * K * vb);
        add(N0 * K * vb);  // partial SpMV sums
        for (int i = 0; i < 3; ++i) add((N0 + 1) * K * vb);  // staging (ABI calls, autotuning)
    }
    if (!((mask >> HPGMX_F64) & 1u))
        for (int i = 0; i < 3; ++i) add((N0 + 1) * K * 8);  // FP64 staging of the residual tuning
    return tot;
}

// ---- argument checks --------------------------------------------------------------------------
void check_ready(hpgmx_ctx *c)
{
    if (c->poisoned) fail(HPGMX_ESTATE, "handle poisoned by an earlier HIP error: " + c->err);
    if (!c->mg_ready) fail(HPGMX_ESTATE, "hpgmx_mg_setup has not been called");
    hip_check(hipSetDevice(c->device), "hipSetDevice");
}

Prec check_dtype(int dtype)
{
    if (dtype < HPGMX_F64 || dtype > HPGMX_BF16_MG) fail(HPGMX_EINVAL, "dtype out of range");
    return (Prec)dtype;
}

void check_level(hpgmx_ctx *c, int level, bool need_coarser)
{
    const int top = (int)c->lv.size() - (need_coarser ? 1 : 0);
    if (level < 0 || level >= top) fail(HPGMX_EINVAL, "level out of range");
}

void check_ptr(const void *p, const char *name)
{
    if (!p) fail(HPGMX_EINVAL, std::string(name) + " is NULL");
}

Prec check_batch_dtype(int dtype)
{
    const Prec p = check_dtype(dtype);
    if (mg16(p)) fail(HPGMX_EINVAL, "the batched solver keeps FP32 multigrid vectors (dtype 0..3)");
    return p;
}

// The batched kernels read int32 column indices.
void check_batch_cols(hpgmx_ctx *c)
{
    if (c->cols16) fail(HPGMX_EINVAL, "batched calls need int32 column indices (HPGMX_COLS_INT32)");
}

void check_nrhs(int nrhs)
{
    if (nrhs < 1 || nrhs > kMaxBatch) fail(HPGMX_EINVAL, "nrhs must be 1..8");
}

void check_solve_desc(const hpgmx_solve_desc *desc)
{
    check_ptr(desc, "desc");
    if (desc->restart < 1 || desc->restart > kMaxRestart) fail(HPGMX_EINVAL, "restart must be 1..63");
    if (desc->max_iters < 0) fail(HPGMX_EINVAL, "max_iters must be >= 0");
    if (!(desc->tol >= 0.0)) fail(HPGMX_EINVAL, "tol must be >= 0");
    check_dtype(desc->inner_dtype);
    if (desc->res_hist_len < 0) fail(HPGMX_EINVAL, "res_hist_len must be >= 0");
}

void fill_tuning(const hpgmx_ctx *c, const Batch &B, Prec p, hpgmx_batch_tuning *out)
{
    std::memset(out, 0, sizeof(*out));
    const int L = (int)c->lv.size();
    for (int k = 0; k < HPGMX_BK_COUNT; ++k)
        for (int l = 0; l < L && l < 8; ++l) {
            if (k == HPGMX_BK_RESTRICT && l + 1 >= L) continue;
            if (k == HPGMX_BK_RESID64 && l > 0) continue;
            out->rhs_per_lane[k][l] = tile_r(c, B, p, k, l);
            out->ms[k][l] = B.tune[p].ms[k][l];
        }
}

template <typename F>
hpgmx_status guarded(hpgmx_ctx *c, F &&f)
{
    if (!c) return HPGMX_EINVAL;
    try {
        return f();
    } catch (const Error &e) {
        c->err = e.msg;
        if (e.st == HPGMX_EHIP) c->poisoned = true;
        return e.st;
    } catch (const std::bad_alloc &) {
        c->err = "host allocation failed";
        return HPGMX_ENOMEM;
    } catch (const std::exception &e) {  // kernel launch errors
        c->err = e.what();
        c->poisoned = true;
        return HPGMX_EHIP;
    }
}

hpgmx_status create(int nx, int ny, int nz, const Stencil &st, double beta, void *hip_stream,
                           hpgmx_handle *out)
{
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return HPGMX_EINVAL;
    const double N = (double)nx * ny * nz;
    if (N >= 2147483647.0) return HPGMX_EINVAL;  // int32 column indices (and entry N)
    for (int t = 0; t < 27; ++t)
        if (!std::isfinite(st.c[t])) return HPGMX_EINVAL;
    if (st.c[13] == 0.0) return HPGMX_EINVAL;    // the smoother divides by the diagonal
    hpgmx_ctx *c = new (std::nothrow) hpgmx_ctx();
    if (!c) return HPGMX_ENOMEM;
    c->prob.nx = nx;
    c->prob.ny = ny;
    c->prob.nz = nz;
    c->prob.beta = beta;
    c->stencil = st;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess || noalloc_setup(c->device) != hipSuccess) {
        delete c;
        return HPGMX_EHIP;
    }
    *out = c;
    return HPGMX_OK;
}

}  // namespace

// =====================================================================================================
extern "C" {

hpgmx_status hpgmx_setup_problem(const hpgmx_problem_desc *desc, void *hip_stream, hpgmx_handle *out)
{
    if (!desc || !out) return HPGMX_EINVAL;
    *out = nullptr;
    if (!std::isfinite(desc->beta)) return HPGMX_EINVAL;
    return create(desc->nx, desc->ny, desc->nz, stencil_from_beta(desc->beta), desc->beta,
                  hip_stream, out);
}

hpgmx_status hpgmx_setup_problem_stencil(const hpgmx_stencil_desc *desc, void *hip_stream,
                                         hpgmx_handle *out)
{
    if (!desc || !out) return HPGMX_EINVAL;
    Stencil st{};
    for (int t = 0; t < 27; ++t) st.c[t] = desc->coef[t];
    return create(desc->nx, desc->ny, desc->nz, st, std::nan(""), hip_stream, out);
}

hpgmx_status hpgmx_workspace_bytes(hpgmx_handle h, const hpgmx_mg_desc *mg, int restart,
                                   unsigned dtype_mask, size_t *bytes)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ptr(mg, "mg");
        check_ptr(bytes, "bytes");
        if (mg->levels < 1 || mg->levels > kMaxLevels) fail(HPGMX_EINVAL, "levels out of range");
        if (restart < 1 || restart > kMaxRestart) fail(HPGMX_EINVAL, "restart out of range");
        *bytes = plan_bytes(h->prob, *mg, restart, dtype_mask & 0x3Fu, h->cols16, h->layout);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_bind_workspace(hpgmx_handle h, void *dev_ptr, size_t bytes)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ptr(dev_ptr, "dev_ptr");
        if (h->mg_ready || h->ws_base || !h->owned.empty())
            fail(HPGMX_ESTATE, "workspace must be bound once, before hpgmx_mg_setup");
        if (((uintptr_t)dev_ptr) % kAlign != 0) fail(HPGMX_EINVAL, "workspace must be 256-byte aligned");
        h->ws_base = (char *)dev_ptr;
        h->ws_size = bytes;
        h->ws_used = 0;
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_set_column_format(hpgmx_handle h, int format)
{
    return guarded(h, [&]() -> hpgmx_status {
        if (h->poisoned) fail(HPGMX_ESTATE, "handle poisoned: " + h->err);
        if (h->mg_ready) fail(HPGMX_ESTATE, "the column format must be chosen before hpgmx_mg_setup");
        if (format != HPGMX_COLS_INT32 && format != HPGMX_COLS_OFFSET16) fail(HPGMX_EINVAL, "unknown column format");
        h->cols16 = format == HPGMX_COLS_OFFSET16;
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_set_layout(hpgmx_handle h, int tile_order, int ell_chunk_log2, int ldq_pad,
                              long long pair_rows, int spmv_in_sweep)
{
    return guarded(h, [&]() -> hpgmx_status {
        if (h->poisoned) fail(HPGMX_ESTATE, "handle poisoned: " + h->err);
        if (h->mg_ready) fail(HPGMX_ESTATE, "the layout must be chosen before hpgmx_mg_setup");
        if (tile_order > kRemapPlanes) fail(HPGMX_EINVAL, "tile_order must be 0..3 (negative: default)");
        if (ell_chunk_log2 > 16) fail(HPGMX_EINVAL, "ell_chunk_log2 must be 0..16 (negative: default)");
        if (ldq_pad > (1 << 20) || (ldq_pad > 0 && ldq_pad % 2))
            fail(HPGMX_EINVAL, "ldq_pad must be even and at most 2^20 (negative: default)");
        const Layout def;
        h->layout.order = tile_order < 0 ? def.order : tile_order;
        h->layout.clog2 = ell_chunk_log2 < 0 ? def.clog2 : ell_chunk_log2;
        h->layout.ldq_pad = ldq_pad < 0 ? def.ldq_pad : ldq_pad;
        h->layout.pair_rows = pair_rows < 0 ? def.pair_rows : pair_rows;
        if (spmv_in_sweep > kSpmvSplitSeparate) fail(HPGMX_EINVAL, "spmv_in_sweep must be 0..3 (negative: default)");
        h->spmv_mode = spmv_in_sweep < 0 ? kSpmvSplit : spmv_in_sweep;
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_mg_setup(hpgmx_handle h, const hpgmx_mg_desc *mg)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ptr(mg, "mg");
        if (h->poisoned) fail(HPGMX_ESTATE, "handle poisoned: " + h->err);
        if (h->mg_ready) fail(HPGMX_ESTATE, "hpgmx_mg_setup already called on this handle");
        if (mg->levels < 1 || mg->levels > kMaxLevels) fail(HPGMX_EINVAL, "levels must be 1..8");
        if (mg->pre_sweeps < 0 || mg->post_sweeps < 0 || mg->coarsest_sweeps < 0)
            fail(HPGMX_EINVAL, "sweep counts must be >= 0");
        if (mg->sweep < HPGMX_GS_FORWARD || mg->sweep > HPGMX_GS_SYMMETRIC)
            fail(HPGMX_EINVAL, "unknown sweep kind");
        const int f = 1 << (mg->levels - 1);
        const hpgmx_problem_desc &pd = h->prob;
        if (pd.nx % f || pd.ny % f || pd.nz % f)
            fail(HPGMX_EINVAL, "every dimension must be divisible by 2^(levels-1)");
        if (pd.nx / f < 2 || pd.ny / f < 2 || pd.nz / f < 2)
            fail(HPGMX_EINVAL, "the coarsest level must be at least 2 in every dimension");
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        h->mg = *mg;
        h->lv.resize(mg->levels);
        int nx = pd.nx, ny = pd.ny, nz = pd.nz;
        std::vector<ColMap> maps(mg->levels);
        int *overflow = (int *)h->dalloc(sizeof(int));
        hip_check(hipMemsetAsync(overflow, 0, sizeof(int), h->stream), "hipMemsetAsync");
        for (int l = 0; l < mg->levels; ++l) {
            Matrix &A = h->lv[l].A;
            A.g = make_geom(nx, ny, nz);
            A.clog2 = h->layout.clog2;
            A.order = h->layout.order;
            A.c16 = h->cols16;
            A.col = h->dalloc((size_t)ell_entries(A.g.N, A.clog2) * (A.c16 ? sizeof(short) : sizeof(int)));
            if (A.c16) {
                A.cmap = (int *)h->dalloc(sizeof(ColMap));
                maps[l] = make_colmap(A.g);
                hip_check(hipMemcpyAsync(A.cmap, &maps[l], sizeof(ColMap), hipMemcpyHostToDevice, h->stream),
                          "hipMemcpyAsync");
            }
            alloc_matrix_prec(h, A, P64);
            alloc_matrix_prec(h, A, P32);
            launch_generate(A, h->stencil, overflow, h->stream);
            nx /= 2; ny /= 2; nz /= 2;
        }
        ensure_common(h);
        if (!h->host_scal) hip_check(hipHostMalloc((void **)&h->host_scal, 256, hipHostMallocDefault), "hipHostMalloc");
        int over = 0;
        hip_check(hipMemcpyAsync(&over, overflow, sizeof(int), hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        if (over)
            fail(HPGMX_EINVAL, "a column offset of the generated matrix does not fit 16 bits (odd level "
                               "extents beyond a few hundred); choose even grid extents");
        h->mg_ready = true;
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_gmres_ir_solve(hpgmx_handle h, const double *b, double *x,
                                  const hpgmx_solve_desc *desc, hpgmx_solve_stats *stats)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_ptr(b, "b");
        check_ptr(x, "x");
        check_solve_desc(desc);
        return solve(h, b, x, desc, stats);
    });
}

hpgmx_status hpgmx_spmv(hpgmx_handle h, int level, int dtype, const void *x, void *y)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, false);
        const Prec p = check_dtype(dtype);
        check_ptr(x, "x");
        check_ptr(y, "y");
        ensure_prec(h, p);
        ensure_tmp(h, p);
        const int vt = vt_of(p);
        const Matrix &A = h->lv[level].A;
        const Prec pv = vprec(p), py = basis_prec(p);  // y is a Krylov vector
        ensure_tmp(h, py);
        void *ty = h->tmp[vt_of(py)][1];
        zero_entry(h, h->tmp[vt][0], A.g.N, pv);
        launch_nat2int(A.g, pv, x, pv, h->tmp[vt][0], h->stream);
        launch_spmv(A, p, h->tmp[vt][0], ty, h->stream);
        launch_int2nat(A.g, py, ty, py, y, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_smooth(hpgmx_handle h, int level, int dtype, int sweep, const void *r, void *z,
                          int zero_guess)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, false);
        const Prec p = check_dtype(dtype);
        if (sweep < HPGMX_GS_FORWARD || sweep > HPGMX_GS_SYMMETRIC) fail(HPGMX_EINVAL, "unknown sweep kind");
        check_ptr(r, "r");
        check_ptr(z, "z");
        ensure_prec(h, p);
        ensure_tmp(h, p);
        const int vt = vt_of(p);
        const Matrix &A = h->lv[level].A;
        const Prec pv = vprec(p);
        zero_entry(h, h->tmp[vt][1], A.g.N, pv);
        launch_nat2int(A.g, pv, r, pv, h->tmp[vt][0], h->stream);
        if (!zero_guess) launch_nat2int(A.g, pv, z, pv, h->tmp[vt][1], h->stream);
        smooth_level(h, level, p, sweep, h->tmp[vt][0], h->tmp[vt][1], zero_guess != 0, 1);
        launch_int2nat(A.g, pv, h->tmp[vt][1], pv, z, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_vcycle(hpgmx_handle h, int dtype, const void *r, void *z)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        const Prec p = check_dtype(dtype);
        check_ptr(r, "r");
        check_ptr(z, "z");
        ensure_prec(h, p);
        ensure_tmp(h, p);
        ensure_level_vectors(h, p);
        const int vt = vt_of(p);
        const Matrix &A = h->lv[0].A;
        const Prec pv = vprec(p);
        zero_entry(h, h->tmp[vt][1], A.g.N, pv);
        launch_nat2int(A.g, pv, r, pv, h->tmp[vt][0], h->stream);
        vcycle(h, 0, p, h->tmp[vt][0], h->tmp[vt][1]);
        launch_int2nat(A.g, pv, h->tmp[vt][1], pv, z, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_restrict_residual(hpgmx_handle h, int level, int dtype, const void *r,
                                     const void *z, void *r_coarse)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, true);
        const Prec p = check_dtype(dtype);
        check_ptr(r, "r");
        check_ptr(z, "z");
        check_ptr(r_coarse, "r_coarse");
        ensure_prec(h, p);
        ensure_tmp(h, p);
        const int vt = vt_of(p);
        const Matrix &A = h->lv[level].A;
        const Geom &gc = h->lv[level + 1].A.g;
        const Prec pv = vprec(p);
        zero_entry(h, h->tmp[vt][1], A.g.N, pv);
        launch_nat2int(A.g, pv, r, pv, h->tmp[vt][0], h->stream);
        launch_nat2int(A.g, pv, z, pv, h->tmp[vt][1], h->stream);
        launch_restrict(A, gc, p, h->tmp[vt][0], h->tmp[vt][1], h->tmp[vt][2], h->stream);
        launch_int2nat(gc, pv, h->tmp[vt][2], pv, r_coarse, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_presmooth_restrict(hpgmx_handle h, int level, int dtype, int sweep, int nsweeps,
                                      const void *r, void *z, void *r_coarse)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, true);
        const Prec p = check_dtype(dtype);
        if (sweep < HPGMX_GS_FORWARD || sweep > HPGMX_GS_SYMMETRIC) fail(HPGMX_EINVAL, "unknown sweep kind");
        if (nsweeps < 0 || nsweeps > 16) fail(HPGMX_EINVAL, "nsweeps must be 0..16");
        check_ptr(r, "r");
        check_ptr(z, "z");
        check_ptr(r_coarse, "r_coarse");
        ensure_prec(h, p);
        ensure_tmp(h, p);
        const int vt = vt_of(p);
        const Matrix &A = h->lv[level].A;
        const Geom &gc = h->lv[level + 1].A.g;
        const Prec pv = vprec(p);
        zero_entry(h, h->tmp[vt][1], A.g.N, pv);
        launch_nat2int(A.g, pv, r, pv, h->tmp[vt][0], h->stream);
        presmooth_restrict(h, level, p, sweep, nsweeps, h->tmp[vt][0], h->tmp[vt][1], h->tmp[vt][2]);
        launch_int2nat(A.g, pv, h->tmp[vt][1], pv, z, h->stream);
        launch_int2nat(gc, pv, h->tmp[vt][2], pv, r_coarse, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_krylov_cycle_get(hpgmx_handle h, int dtype, int *k, double *Q, double *scale, double *Hbar,
                                    double *y)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        const Prec p = check_dtype(dtype);
        check_ptr(k, "k");
        const int kk = h->last_k[p], m = h->last_m[p];
        if (kk < 0 || !h->ctrl) fail(HPGMX_ESTATE, "no single solve with this inner dtype has run");
        *k = kk;
        const Krylov &K = h->kry[p];
        const Geom &g0 = h->lv[0].A.g;
        const Prec bp = basis_prec(p);
        const size_t vb = vec_bytes(bp);
        if (Q)
            for (int j = 0; j <= kk; ++j)
                launch_int2nat(g0, bp, (const char *)K.Q + (size_t)j * K.ldq * vb, P64, Q + (size_t)j * g0.N,
                               h->stream);
        if (scale)
            hip_check(hipMemcpyAsync(scale, h->ctrl->colscale, (size_t)(kk + 1) * 8, hipMemcpyDeviceToHost,
                                     h->stream), "hipMemcpyAsync");
        if (Hbar)
            for (int j = 0; j < kk; ++j)
                hip_check(hipMemcpyAsync(Hbar + (size_t)j * (kk + 1), h->ctrl->Hbar + (size_t)j * (m + 1),
                                         (size_t)(kk + 1) * 8, hipMemcpyDeviceToHost, h->stream),
                          "hipMemcpyAsync");
        if (y)
            hip_check(hipMemcpyAsync(y, h->ctrl->y, (size_t)kk * 8, hipMemcpyDeviceToHost, h->stream),
                      "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_prolong_add(hpgmx_handle h, int level, int dtype, const void *z_coarse, void *z)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, true);
        const Prec p = check_dtype(dtype);
        check_ptr(z_coarse, "z_coarse");
        check_ptr(z, "z");
        ensure_tmp(h, p);
        const int vt = vt_of(p);
        const Geom &gf = h->lv[level].A.g;
        const Geom &gc = h->lv[level + 1].A.g;
        const Prec pv = vprec(p);
        launch_nat2int(gc, pv, z_coarse, pv, h->tmp[vt][0], h->stream);
        launch_nat2int(gf, pv, z, pv, h->tmp[vt][1], h->stream);
        launch_prolong(gf, gc, p, h->tmp[vt][0], h->tmp[vt][1], h->stream);
        launch_int2nat(gf, pv, h->tmp[vt][1], pv, z, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_rhs_from_x(hpgmx_handle h, const double *x, double *b)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_ptr(x, "x");
        check_ptr(b, "b");
        ensure_tmp(h, P64);
        const Matrix &A = h->lv[0].A;
        zero_entry(h, h->tmp[0][0], A.g.N, P64);
        launch_nat2int(A.g, P64, x, P64, h->tmp[0][0], h->stream);
        launch_spmv(A, P64, h->tmp[0][0], h->tmp[0][1], h->stream);
        launch_int2nat(A.g, P64, h->tmp[0][1], P64, b, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_stencil_grad(hpgmx_handle h, const double *lam, const double *x, double *out27)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_ptr(lam, "lam");
        check_ptr(x, "x");
        check_ptr(out27, "out27");
        ensure_common(h);
        ensure_tmp(h, P64);
        const Matrix &A = h->lv[0].A;
        zero_entry(h, h->tmp[0][1], A.g.N, P64);
        launch_nat2int(A.g, P64, lam, P64, h->tmp[0][0], h->stream);
        launch_nat2int(A.g, P64, x, P64, h->tmp[0][1], h->stream);
        launch_stencil_correlation(A, (const double *)h->tmp[0][0], (const double *)h->tmp[0][1],
                                   h->partials, h->ctrl, h->stream);
        hip_check(hipMemcpyAsync(out27, h->ctrl->corr, 27 * sizeof(double), hipMemcpyDeviceToDevice,
                                 h->stream), "hipMemcpyAsync");
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_stencil_grad_noalloc(hpgmx_handle h, const double *lam, const double *x, double *out27)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_ptr(lam, "lam");
        check_ptr(x, "x");
        check_ptr(out27, "out27");
        const Geom &g = h->lv[0].A.g;
        if (red_blocks(g.N) > kMaxRedBlocks) fail(HPGMX_EINVAL, "grid needs more partial sums than the fixed scratch holds");
        launch_stencil_correlation_noalloc(h->device, g, lam, x, out27, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_workspace_bytes_batched(hpgmx_handle h, const hpgmx_mg_desc *mg, int nrhs, int restart,
                                           unsigned dtype_mask, size_t *bytes)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ptr(mg, "mg");
        check_ptr(bytes, "bytes");
        check_nrhs(nrhs);
        if (mg->levels < 1 || mg->levels > kMaxLevels) fail(HPGMX_EINVAL, "levels out of range");
        if (restart < 1 || restart > kMaxRestart) fail(HPGMX_EINVAL, "restart out of range");
        *bytes = plan_batch_bytes(h->prob, *mg, nrhs, restart, dtype_mask & 0xFu, h->layout);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_batch_autotune(hpgmx_handle h, int nrhs, int dtype, hpgmx_batch_tuning *out)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_nrhs(nrhs);
        const Prec p = check_batch_dtype(dtype);
        check_batch_cols(h);
        Batch &B = ensure_batch(h, batch_width(nrhs));
        autotune(h, B, p);
        if (out) fill_tuning(h, B, p, out);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_batch_set_tuning(hpgmx_handle h, int nrhs, int dtype, const hpgmx_batch_tuning *in)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_nrhs(nrhs);
        const Prec p = check_batch_dtype(dtype);
        check_batch_cols(h);
        check_ptr(in, "in");
        const int K = batch_width(nrhs);
        for (int k = 0; k < HPGMX_BK_COUNT; ++k)
            for (int l = 0; l < 8; ++l) {
                const int R = in->rhs_per_lane[k][l];
                if (R != 0 && !batch_shape_ok(K, R))
                    fail(HPGMX_EINVAL, "rhs_per_lane must be 0 or a power of two dividing " + std::to_string(K));
            }
        Batch &B = ensure_batch(h, K);
        BatchTune T{};
        for (int k = 0; k < HPGMX_BK_COUNT; ++k)
            for (int l = 0; l < 8 && l < kMaxLevels; ++l) {
                T.R[k][l] = in->rhs_per_lane[k][l];
                T.ms[k][l] = in->ms[k][l];
            }
        T.set = true;
        B.tune[p] = T;
        h->drop_graphs();
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_batch_get_tuning(hpgmx_handle h, int nrhs, int dtype, hpgmx_batch_tuning *out)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_nrhs(nrhs);
        const Prec p = check_batch_dtype(dtype);
        check_batch_cols(h);
        check_ptr(out, "out");
        Batch &B = ensure_batch(h, batch_width(nrhs));
        fill_tuning(h, B, p, out);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_spmv_batched(hpgmx_handle h, int level, int dtype, int nrhs, const void *X, void *Y)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, false);
        check_nrhs(nrhs);
        const Prec p = check_batch_dtype(dtype);
        check_batch_cols(h);
        check_ptr(X, "X");
        check_ptr(Y, "Y");
        const int K = batch_width(nrhs), vt = vt_of(p);
        Batch &B = ensure_batch(h, K);
        ensure_batch_prec(h, B, p, 0);
        ensure_batch_tmp(h, B, vt);
        const Matrix &A = h->lv[level].A;
        zero_batch_row(h, B.tmp[vt][0], A.g.N, K, p);
        launch_bnat2int(A.g, p, p, K, nrhs, X, B.tmp[vt][0], h->stream);
        launch_bspmv(A, p, K, tile_r(h, B, p, HPGMX_BK_SPMV, level), B.tmp[vt][0], B.tmp[vt][1], h->stream);
        launch_bint2nat(A.g, p, p, K, nrhs, B.tmp[vt][1], Y, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_smooth_batched(hpgmx_handle h, int level, int dtype, int sweep, int nrhs, const void *R,
                                  void *Z, int zero_guess)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, false);
        check_nrhs(nrhs);
        const Prec p = check_batch_dtype(dtype);
        check_batch_cols(h);
        if (sweep < HPGMX_GS_FORWARD || sweep > HPGMX_GS_SYMMETRIC) fail(HPGMX_EINVAL, "unknown sweep kind");
        check_ptr(R, "R");
        check_ptr(Z, "Z");
        const int K = batch_width(nrhs), vt = vt_of(p);
        Batch &B = ensure_batch(h, K);
        ensure_batch_prec(h, B, p, 0);
        ensure_batch_tmp(h, B, vt);
        const Matrix &A = h->lv[level].A;
        zero_batch_row(h, B.tmp[vt][1], A.g.N, K, p);
        launch_bnat2int(A.g, p, p, K, nrhs, R, B.tmp[vt][0], h->stream);
        if (!zero_guess) launch_bnat2int(A.g, p, p, K, nrhs, Z, B.tmp[vt][1], h->stream);
        bsmooth_level(h, B, level, p, sweep, B.tmp[vt][0], B.tmp[vt][1], zero_guess != 0, 1);
        launch_bint2nat(A.g, p, p, K, nrhs, B.tmp[vt][1], Z, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_presmooth_restrict_batched(hpgmx_handle h, int level, int dtype, int sweep, int nsweeps,
                                              int nrhs, const void *R, void *Z, void *R_coarse)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_level(h, level, true);
        check_nrhs(nrhs);
        const Prec p = check_batch_dtype(dtype);
        check_batch_cols(h);
        if (sweep < HPGMX_GS_FORWARD || sweep > HPGMX_GS_SYMMETRIC) fail(HPGMX_EINVAL, "unknown sweep kind");
        if (nsweeps < 0 || nsweeps > 16) fail(HPGMX_EINVAL, "nsweeps must be 0..16");
        check_ptr(R, "R");
        check_ptr(Z, "Z");
        check_ptr(R_coarse, "R_coarse");
        const int K = batch_width(nrhs), vt = vt_of(p);
        Batch &B = ensure_batch(h, K);
        ensure_batch_prec(h, B, p, 0);
        ensure_batch_tmp(h, B, vt);
        const Matrix &A = h->lv[level].A;
        const Geom &gc = h->lv[level + 1].A.g;
        zero_batch_row(h, B.tmp[vt][1], A.g.N, K, p);
        launch_bnat2int(A.g, p, p, K, nrhs, R, B.tmp[vt][0], h->stream);
        bpresmooth_restrict(h, B, level, p, sweep, nsweeps, B.tmp[vt][0], B.tmp[vt][1], B.tmp[vt][2]);
        launch_bint2nat(A.g, p, p, K, nrhs, B.tmp[vt][1], Z, h->stream);
        launch_bint2nat(gc, p, p, K, nrhs, B.tmp[vt][2], R_coarse, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_vcycle_batched(hpgmx_handle h, int dtype, int nrhs, const void *R, void *Z)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_nrhs(nrhs);
        const Prec p = check_batch_dtype(dtype);
        check_batch_cols(h);
        check_ptr(R, "R");
        check_ptr(Z, "Z");
        const int K = batch_width(nrhs), vt = vt_of(p);
        Batch &B = ensure_batch(h, K);
        ensure_batch_prec(h, B, p, 0);
        ensure_batch_tmp(h, B, vt);
        const Matrix &A = h->lv[0].A;
        zero_batch_row(h, B.tmp[vt][1], A.g.N, K, p);
        launch_bnat2int(A.g, p, p, K, nrhs, R, B.tmp[vt][0], h->stream);
        bvcycle(h, B, 0, p, B.tmp[vt][0], B.tmp[vt][1]);
        launch_bint2nat(A.g, p, p, K, nrhs, B.tmp[vt][1], Z, h->stream);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_gmres_ir_solve_batched(hpgmx_handle h, int nrhs, const double *B, double *X,
                                          const hpgmx_solve_desc *desc, hpgmx_solve_stats *stats)
{
    return guarded(h, [&]() -> hpgmx_status {
        check_ready(h);
        check_nrhs(nrhs);
        check_ptr(B, "B");
        check_ptr(X, "X");
        check_solve_desc(desc);
        check_batch_dtype(desc->inner_dtype);
        check_batch_cols(h);
        return bsolve(h, nrhs, B, X, desc, stats);
    });
}

hpgmx_status hpgmx_profile_get(hpgmx_handle h, int kernel, int level, double *total_ms,
                               long long *launches)
{
    return guarded(h, [&]() -> hpgmx_status {
        if (kernel < 0 || kernel >= HPGMX_K_COUNT || level < 0 || level >= kMaxLevels)
            fail(HPGMX_EINVAL, "kernel or level out of range");
        if (total_ms) *total_ms = h->prof_ms[kernel][level];
        if (launches) *launches = h->prof_n[kernel][level];
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_stream_copy(hpgmx_handle h, const void *src, void *dst, size_t bytes, int reps,
                               double *ms)
{
    return guarded(h, [&]() -> hpgmx_status {
        if (h->poisoned) fail(HPGMX_ESTATE, "handle poisoned: " + h->err);
        check_ptr(src, "src");
        check_ptr(dst, "dst");
        check_ptr(ms, "ms");
        if (bytes == 0 || bytes % 16 || reps < 1) fail(HPGMX_EINVAL, "bytes must be a positive multiple of 16, reps >= 1");
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
        launch_copy(src, dst, bytes, h->stream);  // warm-up
        hip_check(hipEventRecord(e0, h->stream), "hipEventRecord");
        for (int i = 0; i < reps; ++i) launch_copy(src, dst, bytes, h->stream);
        hip_check(hipEventRecord(e1, h->stream), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float t = 0.f;
        hip_check(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
        *ms = t / reps;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return HPGMX_OK;
    });
}

hpgmx_status hpgmx_destroy(hpgmx_handle h)
{
    if (!h) return HPGMX_EINVAL;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (auto &e : h->evpool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    h->drop_graphs();
    if (h->own) {
        (void)hipStreamSynchronize(h->own);
        (void)hipStreamDestroy(h->own);
        (void)hipEventDestroy(h->ev_in);
        (void)hipEventDestroy(h->ev_out);
    }
    for (void *p : h->owned) (void)hipFree(p);
    if (h->host_scal) (void)hipHostFree(h->host_scal);
    for (auto &e : h->ev_scal)
        if (e) (void)hipEventDestroy(e);
    for (auto &kv : h->batches)
        if (kv.second.host_scal) (void)hipHostFree(kv.second.host_scal);
    delete h;
    return HPGMX_OK;
}

const char *hpgmx_last_error(hpgmx_handle h)
{
    if (!h) return "invalid handle";
    return h->err.c_str();
}

}  // extern "C"
