"""Independent constructions used to pin the oracle (test-side only).

Nothing here calls the oracle or the HIP library.  The operator is built from
Kronecker products of 1-D tridiagonal matrices, Gauss-Seidel is written as the
two triangular solves of the splitting (D+L) y = r - U z / (D+U) z' = r - L y
on the colour-permuted matrix, and the V-cycle is composed from those pieces
with an explicit selection matrix for the injection.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular


def dims3(d):
    return (d, d, d) if isinstance(d, int) else tuple(int(v) for v in d)


def kron_matrix(d, beta=0.5, faces_only=False):
    """27-point operator: 27 I - Tz (x) Ty (x) Tx with T = tridiag(1, 1, 1).

    The x factor carries the nonsymmetric shift: sub-diagonal (neighbour at
    i-1) 1+beta, super-diagonal 1-beta, so the entries become -1-beta and
    -1+beta.  With faces_only the shift is applied only to the face pair.
    """
    nx, ny, nz = dims3(d)
    n = nx * ny * nz

    def tri(m, sub=1.0, sup=1.0):
        return sp.diags([np.full(m - 1, sub), np.ones(m), np.full(m - 1, sup)], [-1, 0, 1])

    if faces_only:
        A = 27.0 * sp.identity(n) - sp.kron(tri(nz), sp.kron(tri(ny), tri(nx)))
        shift = sp.diags([np.ones(nx - 1), -np.ones(nx - 1)], [-1, 1])
        A = A - beta * sp.kron(sp.identity(nz), sp.kron(sp.identity(ny), shift))
    else:
        A = 27.0 * sp.identity(n) - sp.kron(tri(nz), sp.kron(tri(ny), tri(nx, 1.0 + beta, 1.0 - beta)))
    return sp.csr_matrix(A)


def grid_coords(d):
    nx, ny, nz = dims3(d)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def colour_of(d):
    i, j, k = grid_coords(d)
    return (i & 1) + 2 * (j & 1) + 4 * ((k + 1) & 1)


def colour_perm(d):
    return np.argsort(colour_of(d), kind="stable")


def injection_matrix(d):
    """R with (R v)_I = v at fine point (2I, 2J, 2K)."""
    nx, ny, nz = dims3(d)
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    K, J, I = np.meshgrid(np.arange(cz), np.arange(cy), np.arange(cx), indexing="ij")
    fine = (2 * I + nx * (2 * J + ny * 2 * K)).ravel()
    nc = cx * cy * cz
    return sp.csr_matrix((np.ones(nc), (np.arange(nc), fine)), shape=(nc, nx * ny * nz))


def gs_triangular(A, perm, r, z, sweep):
    """Gauss-Seidel in the colour-permuted ordering as triangular solves."""
    Ap = sp.csr_matrix(A[perm][:, perm])
    D = sp.diags(Ap.diagonal())
    L = sp.tril(Ap, -1, format="csr")
    U = sp.triu(Ap, 1, format="csr")
    rp, zp = r[perm], z[perm].copy()
    if sweep in (0, 2):
        zp = spsolve_triangular(sp.csr_matrix(D + L), rp - U @ zp, lower=True)
    if sweep in (1, 2):
        zp = spsolve_triangular(sp.csr_matrix(D + U), rp - L @ zp, lower=False)
    out = np.empty_like(zp)
    out[perm] = zp
    return out


def keep(v):
    return v


def fl32(v):
    """Round to the nearest binary32 (ties to even) and widen back: numpy's
    float64 -> float32 conversion is the IEEE one."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_format(v, p, emin, maxv):
    """Round to the nearest value (ties to even) of a binary format with p
    significand bits (the leading one included), smallest normal exponent
    emin and largest finite value maxv, straight from float64 (IEEE 754
    round-to-nearest-even; the quantum is fixed at 2^(emin-p+1) below the
    normal range, and values rounding above maxv overflow)."""
    v = np.asarray(v, dtype=np.float64)
    _, e = np.frexp(v)
    lead = np.maximum(e - 1, emin)
    q = lead - (p - 1)
    r = np.ldexp(np.rint(np.ldexp(v, -q)), q)
    r = np.where(np.abs(r) > maxv, np.copysign(np.inf, v), r)
    return np.where(v == 0.0, v, r)


def fl16(v):
    """IEEE binary16 rounding (ties to even), widened back to float64."""
    return round_format(v, 11, -14, 65504.0)


def flbf16(v):
    """bfloat16 rounding (8-bit significand, binary32's exponent range)."""
    return round_format(v, 8, -126, float.fromhex("0x1.fep127"))


def vcycle_ref(d, r, levels, pre=1, post=1, coarsest=1, sweep=0, beta=0.5, faces_only=False,
               store=keep, coef=None):
    """The V-cycle composed from the pieces above.  `store` is applied to
    every vector the cycle keeps (after each sweep, the restricted residual,
    the corrected z): identity for the FP64 method, fl32 for binary32
    storage of the multigrid work vectors.  With `coef` every level uses
    that 27-entry stencil table instead of the beta family."""
    d = dims3(d)
    A = kron_matrix(d, beta, faces_only) if coef is None else stencil_matrix(d, coef)
    perm = colour_perm(d)
    z = np.zeros(A.shape[0])
    if levels == 1:
        for _ in range(coarsest):
            z = store(gs_triangular(A, perm, r, z, sweep))
        return z
    for _ in range(pre):
        z = store(gs_triangular(A, perm, r, z, sweep))
    R = injection_matrix(d)
    rc = store(R @ (r - A @ z))
    zc = vcycle_ref((d[0] // 2, d[1] // 2, d[2] // 2), rc, levels - 1, pre, post, coarsest,
                    sweep, beta, faces_only, store, coef)
    z = store(z + R.T @ zc)
    for _ in range(post):
        z = store(gs_triangular(A, perm, r, z, sweep))
    return z


def shift_matrix(d, di, dj, dk):
    """(S x)_i = x at the grid neighbour (i+di, j+dj, k+dk), 0 outside the grid."""
    nx, ny, nz = dims3(d)

    def s1(m, delta):
        return sp.diags([np.ones(m - abs(delta))], [delta])

    return sp.csr_matrix(sp.kron(s1(nz, dk), sp.kron(s1(ny, dj), s1(nx, di))))


def stencil_matrix(d, coef27):
    """sum over the 27 offsets of coef * shift (slot s = 9(dk+1) + 3(dj+1) + (di+1))."""
    A = None
    for s in range(27):
        di, dj, dk = s % 3 - 1, (s // 3) % 3 - 1, s // 9 - 1
        term = coef27[s] * shift_matrix(d, di, dj, dk)
        A = term if A is None else A + term
    return sp.csr_matrix(A)
