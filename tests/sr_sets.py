"""Segmental-refinement FMG restated with whole-level arrays and region masks.

A brute-force second formulation for tiny grids, used only to check the
oracle's bookkeeping.  Where the oracle stores each segment as a box and loops
over index ranges, this module keeps every segment's data on a full padded
level array (NaN wherever the segment stores nothing) and builds each region
of Sec. 4 of the paper from its set definition:

    genuine     V_p                              a cube of the segment grid
    compute     C_p   = dilate(V_p, J) & domain  (Chebyshev dilation)
    ghosts      G_p   = dilate(C_p, 1) & ~C_p,   GSR = G & domain
    support     F_{l-1} = coarse cells whose children all lie in C_l

Operators are applied to whole arrays with numpy slicing and the results are
kept only on the region mask; cells of one colour depend only on the other
colour, so a vectorised half-sweep is an exact Gauss-Seidel half-sweep.  Any
NaN read by a kept cell reaches the result, so a footprint that leaves a
segment's storage shows up as NaN.
"""
import numpy as np
from scipy import ndimage

_BALL = np.ones((3, 3, 3), dtype=bool)


def _padded(n, fill=0.0):
    return np.full((n + 2,) * 3, fill)


def _domain(n):
    m = np.zeros((n + 2,) * 3, dtype=bool)
    m[1:-1, 1:-1, 1:-1] = True
    return m


def _box(n, a, b):
    """mask of cells with a_d <= index_d < b_d (indices -1..n), order (x,y,z)"""
    m = np.zeros((n + 2,) * 3, dtype=bool)
    m[a[2] + 1:b[2] + 1, a[1] + 1:b[1] + 1, a[0] + 1:b[0] + 1] = True
    return m


def _dilate(mask, r):
    return ndimage.binary_dilation(mask, structure=_BALL, iterations=r) if r > 0 else mask.copy()


def _colour(n, col):
    i = np.arange(-1, n + 1)
    s = i[:, None, None] + i[None, :, None] + i[None, None, :]
    return (s % 2) == col


def _boundary_count(n):
    """number of faces of each interior cell on the domain boundary"""
    d = _domain(n).astype(np.int64)
    b = np.zeros_like(d)
    inner = (slice(1, -1),) * 3
    for ax in range(3):
        for sh in (-1, 1):
            b[inner] += 1 - np.roll(d, sh, axis=ax)[inner]
    return b


def _nbsum(U, n):
    """sum over the 6 neighbours that lie inside the domain (interior cells)"""
    Z = np.where(_domain(n), U, 0.0)
    out = np.full_like(U, np.nan)
    c = slice(1, -1)
    out[c, c, c] = (Z[:-2, c, c] + Z[2:, c, c] + Z[c, :-2, c] + Z[c, 2:, c]
                    + Z[c, c, :-2] + Z[c, c, 2:])
    return out


def apply_L(U, n):
    b = _boundary_count(n)
    return (_nbsum(U, n) - (6 + b) * U) * float(n * n)


def gs_half(U, R, n, region, col):
    b = _boundary_count(n)
    new = (_nbsum(U, n) - R / float(n * n)) / (6 + b)
    m = region & _colour(n, col)
    U[m] = new[m]


def smooth(U, R, n, region, nu):
    for _ in range(nu):
        gs_half(U, R, n, region, 0)
        gs_half(U, R, n, region, 1)


def restrict(U, n):
    """padded fine -> padded coarse (interior = mean of 8 children)"""
    nc = n // 2
    v = U[1:-1, 1:-1, 1:-1].reshape(nc, 2, nc, 2, nc, 2)
    out = _padded(nc, np.nan)
    out[1:-1, 1:-1, 1:-1] = v.mean(axis=(1, 3, 5))
    return out


def coarse_of(mask_fine, n):
    nc = n // 2
    v = mask_fine[1:-1, 1:-1, 1:-1].reshape(nc, 2, nc, 2, nc, 2)
    out = np.zeros((nc + 2,) * 3, dtype=bool)
    out[1:-1, 1:-1, 1:-1] = v.all(axis=(1, 3, 5))
    return out


def prolong(Uc, nc):
    """padded coarse -> padded fine, each child takes its parent's value;
    fine ghost index -1 has parent -1, fine index 2nc has parent nc"""
    n = 2 * nc
    idx = np.arange(-1, n + 1) // 2 + 1  # padded coarse position of each padded fine position
    return Uc[np.ix_(idx, idx, idx)]


def _interp_axis(A, axis):
    """1D FMG interpolation along one axis of an interior (unpadded) array"""
    A = np.moveaxis(A, axis, 0)
    nc = A.shape[0]
    P = np.concatenate([-A[:1], A, -A[-1:]], axis=0)  # odd reflection at the walls
    out = np.empty((2 * nc,) + A.shape[1:])
    out[0::2] = 0.75 * P[1:-1] + 0.25 * P[:-2]
    out[1::2] = 0.75 * P[1:-1] + 0.25 * P[2:]
    return np.moveaxis(out, 0, axis)


def interp(Uc, nc):
    """padded coarse -> padded fine (interior only), trilinear, odd reflection"""
    A = Uc[1:-1, 1:-1, 1:-1]
    for ax in range(3):
        A = _interp_axis(A, ax)
    out = _padded(2 * nc, np.nan)
    out[1:-1, 1:-1, 1:-1] = A
    return out


def coarse_exact(R, n):
    """dense solve of the level-0 system, matrix built column by column"""
    m = n ** 3
    A = np.zeros((m, m))
    for c in range(m):
        unit = np.zeros(m)
        unit[c] = 1.0
        e = _padded(n)
        e[1:-1, 1:-1, 1:-1] = unit.reshape(n, n, n)
        A[:, c] = apply_L(e, n)[1:-1, 1:-1, 1:-1].reshape(-1)
    U = _padded(n)
    U[1:-1, 1:-1, 1:-1] = np.linalg.solve(A, R[1:-1, 1:-1, 1:-1].reshape(-1)).reshape(n, n, n)
    return U


class _Global:
    def __init__(self, f, L):
        N = f.shape[0]
        self.n = [N >> (L - 1 - l) for l in range(L)]
        self.f = [None] * L
        F = _padded(N)
        F[1:-1, 1:-1, 1:-1] = f
        self.f[L - 1] = F
        for l in range(L - 1, 0, -1):
            self.f[l - 1] = restrict(self.f[l], self.n[l])
        self.u = [_padded(n) for n in self.n]
        self.t = [None] * L
        self.rhs = [None] * L


def vcycle(G, l, R, sw):
    n = G.n[l]
    D = _domain(n)
    if l == 0:
        G.u[0] = coarse_exact(R, n)
        return
    U = G.u[l]
    smooth(U, R, n, D, sw[0])
    res = R - apply_L(U, n)
    G.u[l - 1] = restrict(U, n)
    G.t[l - 1] = G.u[l - 1].copy()
    G.rhs[l - 1] = restrict(res, n) + apply_L(G.u[l - 1], G.n[l - 1])
    vcycle(G, l - 1, G.rhs[l - 1], sw)
    corr = prolong(G.u[l - 1] - G.t[l - 1], G.n[l - 1])
    U[D] += corr[D]
    smooth(U, R, n, D, sw[1])


def fmg(f, L, alpha=1, nu1=2, nu2=2, top=None, G=None):
    G = G or _Global(f, L)
    top = L - 1 if top is None else top
    G.u[0] = coarse_exact(G.f[0], G.n[0])
    for l in range(1, top + 1):
        D = _domain(G.n[l])
        G.u[l] = interp(G.u[l - 1], G.n[l - 1])
        G.u[l][~D] = 0.0
        smooth(G.u[l], G.f[l], G.n[l], D, alpha)
        vcycle(G, l, G.f[l], (nu1, nu2))
    return G


def srfmg(f, L, K, S, J, alpha=1, nu1=2, nu2=2):
    """Figs. 5 and 6 with masks; J finest first.  Returns u (N^3)."""
    N = f.shape[0]
    G = _Global(f, L)
    T = L - 1 - K
    fmg(f, L, alpha, nu1, nu2, top=T, G=G)
    sw = (nu1, nu2)
    segs = [(px, py, pz) for pz in range(S) for py in range(S) for px in range(S)]
    Jl = {l: J[L - 1 - l] for l in range(T + 1, L)}
    reg = {}
    for l in range(T, L):
        n = G.n[l]
        g = n // S
        D = _domain(n)
        for p in segs:
            V = _box(n, [q * g for q in p], [(q + 1) * g for q in p])
            if l == T:
                reg[(l, p)] = dict(V=V)
                continue
            C = _dilate(V, Jl[l]) & D
            Gh = _dilate(C, 1) & ~C
            reg[(l, p)] = dict(V=V, C=C, GSR=Gh & D, F=None)
        if l > T + 1:
            for p in segs:
                reg[(l - 1, p)]["F"] = coarse_of(reg[(l, p)]["C"], n)
    U = {(l, p): _padded(G.n[l], np.nan) for l in range(T + 1, L) for p in segs}
    Tt = {}
    R = {}

    def rhs_of(l, top, p):
        return G.f[l] if l == top else R[(l, p)]

    def vsr(l, top):
        n = G.n[l]
        res = {}
        for p in segs:
            r = reg[(l, p)]
            smooth(U[(l, p)], rhs_of(l, top, p), n, r["C"], sw[0])
            res[p] = np.where(r["C"], rhs_of(l, top, p) - apply_L(U[(l, p)], n), np.nan)
        if l - 1 > T:
            nc = G.n[l - 1]
            for p in segs:
                rc = reg[(l - 1, p)]
                F = rc["F"]
                Ru = restrict(U[(l, p)], n)
                U[(l - 1, p)][F] = Ru[F]
                Tt[(l - 1, p)] = U[(l - 1, p)].copy()
                Lu = apply_L(U[(l - 1, p)], nc)
                rr = np.where(F, restrict(res[p], n), 0.0)
                Rn = np.full_like(Lu, np.nan)
                Rn[rc["C"]] = (rr + Lu)[rc["C"]]
                R[(l - 1, p)] = Rn
            vsr(l - 1, top)
            for p in segs:
                r = reg[(l, p)]
                rng = r["C"] | r["GSR"]
                corr = prolong(U[(l - 1, p)] - Tt[(l - 1, p)], nc)
                U[(l, p)][rng] += corr[rng]
        else:
            nT = G.n[T]
            uT = G.u[T].copy()
            rT = _padded(nT)
            for p in segs:
                Vt = reg[(T, p)]["V"]
                uT[Vt] = restrict(U[(l, p)], n)[Vt]
                rT[Vt] = restrict(res[p], n)[Vt]
            G.u[T] = uT
            tT = uT.copy()
            rhsT = rT + apply_L(uT, nT)
            rhsT[~_domain(nT)] = 0.0
            vcycle(G, T, rhsT, sw)
            for p in segs:
                r = reg[(l, p)]
                rng = r["C"] | r["GSR"]
                corr = prolong(G.u[T] - tT, nT)
                U[(l, p)][rng] += corr[rng]
        for p in segs:
            smooth(U[(l, p)], rhs_of(l, top, p), n, reg[(l, p)]["C"], sw[1])

    for l in range(T + 1, L):
        n = G.n[l]
        for p in segs:
            r = reg[(l, p)]
            src = G.u[T] if l - 1 == T else U[(l - 1, p)]
            P = interp(src, G.n[l - 1])
            rng = r["C"] | r["GSR"]
            U[(l, p)][rng] = P[rng]
            smooth(U[(l, p)], G.f[l], n, r["C"], alpha)
        vsr(l, l)
    out = np.full((N + 2,) * 3, np.nan)
    for p in segs:
        V = reg[(L - 1, p)]["V"]
        out[V] = U[(L - 1, p)][V]
    return out[1:-1, 1:-1, 1:-1]
