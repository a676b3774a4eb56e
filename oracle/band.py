"""The computational band Omega(S) and the interior-boundary sets.

Grid (Sec. 3.2): nodes x_k = k / N for integer k in Z^d, spacing h = 1/N.
Band (eq. bandwidth): Omega(S) = { x_k : ||x_k - cp_S(x_k)|| <= r } with
r = sqrt((d-1)((p+1)/2)^2 + (q+(p+1)/2)^2) / N; p = 3 (cubic interpolation)
and q = 1 (the 2d+1-point Laplacian) give sqrt(13)/N in R^2, sqrt(17)/N in R^3.

PDE DOFs are the band nodes in lexicographic order of k (last axis slowest:
sorted by (k_z, k_y, k_x)).  The set is found by scanning a bounding box of S;
``bfs_band`` is Algorithm 1 (breadth-first search from one band node over the
2d face neighbours) and serves to check the scan.

Interior boundary C (Sec. 4.1, 4.6):
  Omega(C) = { x_i in Omega(S) : ||x_i - cp_C(x_i)|| <= r }   (BC DOFs)
  K(C)     = { x_i in Omega(S) : ||x_i - cp_C(x_i)|| <  2r }  (check region)
Side vector (eq. cpdiff, Sec. 4.2): v_i = cp_S(x_i) - cp_C(x_i), replaced by
tau * o_C(cp_C(x_i)) when ||v_i|| < tau = 0.1 h^2 (the on-C tie rule).
"""


import numpy as np

from .geometry import band_radius_factor


def grid_h(N):
    return 1.0 / N


def band_radius(N, dim, p=3, q=1):
    return np.sqrt(band_radius_factor(dim, p, q)) / N


def node_coords(K, N):
    """x_k = k / N, one correctly rounded division per coordinate."""
    return K.astype(np.float64) / float(N)


def _dist(X, CP):
    D = X - CP
    return np.sqrt(dot_rows(D, D))


def bounding_box(surface, N, r):
    """Integer index box [lo, hi] (inclusive) containing every node within r
    of the surface, with one node of margin."""
    lo = np.floor((surface.c - surface.extent - r) * N).astype(np.int64) - 1
    hi = np.ceil((surface.c + surface.extent + r) * N).astype(np.int64) + 1
    return lo, hi


def scan_band(surface, N, p=3, q=1, r=None):
    """Omega(S) by a bounding-box scan.  Returns (K, CP): integer coordinates
    (n, d) in lexicographic order and the stored closest points (n, d)."""
    d = surface.dim
    if r is None:
        r = band_radius(N, d, p, q)
    lo, hi = bounding_box(surface, N, r)
    axes = [np.arange(lo[a], hi[a] + 1, dtype=np.int64) for a in range(d)]
    Ks, CPs = [], []
    # iterate over the slowest axis to bound memory
    for k_last in axes[-1]:
        grids = np.meshgrid(*axes[:-1], indexing="ij")
        sub = np.stack([g.ravel() for g in grids], axis=1)
        K = np.concatenate([sub, np.full((sub.shape[0], 1), k_last)], axis=1)
        X = node_coords(K, N)
        CP = surface.cp(X)
        dist = _dist(X, CP)
        keep = dist <= r
        if keep.any():
            Ks.append(K[keep])
            CPs.append(CP[keep])
    K = np.concatenate(Ks)
    CP = np.concatenate(CPs)
    order = np.lexsort(tuple(K[:, a] for a in range(d)))
    return K[order], CP[order]


def bfs_band(surface, N, k0, p=3, q=1, r=None):
    """The band as Algorithm 1 defines it: the nodes within r of S that are
    connected to the seed node k0 through face neighbours, with cp_S
    evaluated only at nodes the search reaches.  Grown one breadth-first
    layer at a time: the next layer is every not yet seen face neighbour of
    the current layer that lies within r.  Only for small grids.  Returns the
    set of integer coordinate tuples."""
    d = surface.dim
    if r is None:
        r = band_radius(N, d, p, q)
    k0 = tuple(int(v) for v in k0)
    X0 = node_coords(np.array([k0]), N)
    assert _dist(X0, surface.cp(X0))[0] <= r, "the search must start at a band node"
    steps = [tuple(s if a == b else 0 for b in range(d)) for a in range(d) for s in (-1, 1)]
    band, seen, layer = {k0}, {k0}, [k0]
    while layer:
        fresh = sorted({tuple(k[b] + o[b] for b in range(d)) for k in layer for o in steps}
                       - seen)
        if not fresh:
            break
        seen.update(fresh)
        X = node_coords(np.array(fresh), N)
        keep = _dist(X, surface.cp(X)) <= r
        layer = [k for k, ok in zip(fresh, keep) if ok]
        band.update(layer)
    return band


class IndexMap:
    """Dense lookup from integer coordinates to PDE DOF index (-1 if absent)
    over the bounding box of the band."""

    def __init__(self, K):
        self.lo = K.min(axis=0) - 8
        self.hi = K.max(axis=0) + 8
        self.shape = tuple((self.hi - self.lo + 1).tolist())
        self.table = np.full(self.shape, -1, dtype=np.int64)
        self.table[tuple((K - self.lo).T)] = np.arange(K.shape[0])

    def __call__(self, Kq):
        Kq = np.asarray(Kq)
        rel = Kq - self.lo
        ok = np.all((rel >= 0) & (rel < np.array(self.shape)), axis=-1)
        out = np.full(Kq.shape[:-1], -1, dtype=np.int64)
        relc = np.where(ok[..., None], rel, 0)
        vals = self.table[tuple(np.moveaxis(relc, -1, 0))]
        out[ok] = vals[ok]
        return out


class IBCSets:
    """Per-C sets of Sec. 4.1 and 4.6 and the side vectors of Sec. 4.2."""

    def __init__(self, curve, K, CP, N, r, tau):
        X = node_coords(K, N)
        CPC = curve.cp(X)
        dC = _dist(X, CPC)
        self.curve = curve
        self.in_omega = dC <= r            # Omega(C)
        self.in_check = dC < 2.0 * r       # K(C)
        if hasattr(curve, "at_boundary"):
            # open curve: no BC DOFs and no stencil modification where cp_C is
            # an endpoint (Omega(dC), eq. IBC_boundary_set)
            end = curve.at_boundary(X)
            self.in_omega &= ~end
            self.in_check &= ~end
        self.omega_nodes = np.nonzero(self.in_omega)[0]   # lexicographic
        self.cpc = CPC
        V = CP - CPC
        nv = np.sqrt(dot_rows(V, V))
        on_c = nv < tau
        O = curve.orient(CPC)
        V[on_c] = tau * O[on_c]
        self.v = V
        self.on_c = on_c & self.in_check
        # own side of a node: sign of v . o_C (0 counts as +)
        side_dot = dot_rows(V, O)
        self.side = np.where(side_dot < 0.0, -1, 1)


def dot_rows(A, B):
    """Row-wise dot product in the written order ((a0 b0 + a1 b1) + a2 b2)."""
    s = A[..., 0] * B[..., 0] + A[..., 1] * B[..., 1]
    for a in range(2, A.shape[-1]):
        s = s + A[..., a] * B[..., a]
    return s
