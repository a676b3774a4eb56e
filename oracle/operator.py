"""Discretisation: interpolation stencils with interior-boundary swaps, the
finite-difference Laplacian, BC-DOF rows, explicit E and L (Sec. 5.3) and the
system A = m I + n [diag(L) + (L - diag(L)) E] (Sec. 5.4).

Unknown vector (Sec. 4.1): PDE DOFs 0..N_S-1 (band nodes, lexicographic), then
BC DOFs N_S..N_S+N_C-1 (the nodes of Omega(C), lexicographic within each C,
concatenated over the C's in the order given).

Interpolation (eq. interp-stencil): for a query y the stencil is the (p+1)^d
nodes b + {0..p}^d; cubic (p = 3): b = floor(y N) - 1 per axis, t = y N -
floor(y N); quadratic (p = 2, Sec. 7): the nearest nodes, b = floor(y N +
1/2) - 1, t = y N - (b + 1).  The weights are the tensor product of 1-D
barycentric-Lagrange weights (Berrut and Trefethen's second form) on the
nodes 0..p at the query 1 + t.

Laplacian (eq. FD-stencil): weight -2d N^2 on the centre and N^2 on each face
neighbour in the band; a neighbour outside the band is dropped.

Band: the tube of eq. (bandwidth), or the stencil set (Sec. 5.1 cites it as
keeping only the grid points interpolation and FD stencils need): the nodes
of the DOFs that some interpolation stencil of the tube system uses, and the
FD neighbours of those DOFs' rows.  The rows of the stencil-referenced DOFs
are unchanged, so on them the solution is the tube's.

Interior boundaries (Sec. 4.3), with the readings below:
  * PDE row i in K(C): an interpolation member or FD neighbour j in Omega(C)
    is replaced by its BC DOF alpha(j) when d*_i . v_j < 0 (eq.
    stencil-crossing-test), d*_i = v_i.  A zero dot means "same side".
  * BC row alpha at node j: FD neighbours restricted to Omega(C); neighbour
    beta stays a BC DOF unless d*_alpha . v_beta < 0, then it becomes the PDE
    DOF (eq. FD-crossing-test), d*_alpha = v_j.
  * BC row E, Dirichlet (Sec. 4.3 last paragraph): first order u_alpha =
    g_alpha (no linear part); second order u_alpha = 2 g_alpha - u(cpbar_C)
    with cpbar_C(x) = cp_S(2 cp_C(x) - x) (eq. cpc-bar), the mirror stencil's
    member m stays a BC DOF when on the director's side and in Omega(C), and
    is the PDE DOF otherwise.
  * BC row E, zero Neumann (Sec. 4.3, eq. IBC-1st-order-Neumann and eq.
    cpc-bar): u_alpha = u(y) interpolated at y = cp_C(x) (first order) or
    y = cpbar_C(x) (second order), members chosen as for the Dirichlet mirror
    row, no constant.
  * Each side of a C carries its own condition (Sec. 4.2, mixed IBCs).  A BC
    DOF whose node lies on side s stands in for side -s (a stencil of side -s
    swaps to it), so it takes the condition of side -s.
  * Every row (PDE and BC) uses the stabilised form M = diag L + (L - diag L)E;
    the Dirichlet constants e of E move to the right-hand side:
    A u = f - n (L - diag L) e.
"""

import numpy as np
import scipy.sparse as sp

from .band import (IBCSets, IndexMap, band_radius, dot_rows, node_coords,
                   scan_band)


class StencilHole(RuntimeError):
    """A stencil member is not a band node (the band is too narrow)."""


def stencil_set_nodes(tube):
    """Stencil set of a tube system (Sec. 5.1): a boolean over its PDE nodes
    (lexicographic) that keeps every node whose PDE or BC DOF is a column of
    E (a member of some interpolation stencil), and every node carrying a DOF
    that is an FD neighbour of such a DOF's row."""
    used = np.zeros(tube.n, dtype=bool)
    used[tube.E.tocsr().indices] = True
    rows = np.nonzero(used)[0]
    need = used.copy()
    need[tube.L_off.tocsr()[rows].indices] = True
    keep = need[:tube.n_s].copy()
    keep[tube.bc_node[need[tube.n_s:]]] = True
    return keep


def lagrange_weights_1d(t, p=3):
    """Barycentric-Lagrange weights of degree p on nodes z = 0, 1, .., p at
    xi = 1 + t.  Barycentric weights for equispaced nodes: lam_j = (-1)^j
    C(p, j).  Returns an (n, p + 1) array; exact node hits give the unit
    vector."""
    from math import comb
    t = np.asarray(t, dtype=np.float64)
    xi = 1.0 + t
    lam = np.array([(-1.0) ** j * comb(p, j) for j in range(p + 1)])
    diff = xi[:, None] - np.arange(p + 1.0)[None, :]
    hit = diff == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        q = lam[None, :] / diff
        W = q / np.sum(q, axis=1, keepdims=True)
    rows = hit.any(axis=1)
    if rows.any():
        W[rows] = hit[rows].astype(np.float64)
    return W


def stencil(Y, N, dim, p=3):
    """Base node b (n, d) and tensor weights (n, (p+1)^d) for query points Y:
    the (p+1)^d nodes b + {0..p}^d around y N.  Cubic (p = 3): b = floor(y N)
    - 1, the query at b + 1 + t with t in [0, 1).  Quadratic (p = 2): the
    nodes nearest to y N, b = floor(y N + 1/2) - 1, t in [-1/2, 1/2).
    Member o has offset (o % (p+1), (o // (p+1)) % (p+1), o // (p+1)^2),
    first axis fastest."""
    S = Y * float(N)
    F = np.floor(S) if p == 3 else np.floor(S + 0.5)
    base = F.astype(np.int64) - 1
    T = S - F
    Wax = [lagrange_weights_1d(T[:, a], p) for a in range(dim)]
    m = p + 1
    if dim == 2:
        W = (Wax[1][:, :, None] * Wax[0][:, None, :]).reshape(-1, m * m)
    else:
        W = (Wax[2][:, :, None, None] * Wax[1][:, None, :, None]
             * Wax[0][:, None, None, :]).reshape(-1, m ** 3)
    return base, W


def member_offsets(dim, p=3):
    m = p + 1
    o = np.arange(m ** dim)
    cols = [o % m, (o // m) % m]
    if dim == 3:
        cols.append(o // (m * m))
    return np.stack(cols, axis=1)


def face_offsets(dim):
    out = []
    for a in range(dim):
        for s in (-1, 1):
            e = [0] * dim
            e[a] = s
            out.append(e)
    return np.array(out, dtype=np.int64)


class CPMSystem:
    """The discrete CPM system for one surface, one grid and a list of
    interior boundaries; bc_types[c] = (condition of side +1, of side -1),
    each "dirichlet" or "neumann" (default: Dirichlet on both sides).

    Attributes
      K, CP        PDE nodes (lexicographic) and their stored cp_S
      n_s, n_c     numbers of PDE and BC DOFs
      E, L         (n, n) CSR, n = n_s + n_c, linear parts only
      e_coef       (n_c,) multiplier of g in the constant of E (Dirichlet:
                   1 or 2 by order; Neumann: 0)
      bc_kind      (n_c,) condition of each BC DOF (0 Dirichlet, 1 Neumann)
      bc_node      (n_c,) PDE DOF of the node each BC DOF sits on
      bc_curve     (n_c,) index of the C each BC DOF belongs to
      bc_cpc       (n_c, d) cp_C of the node (where the Dirichlet value is read)
      bc_side      (n_c,) own side of the node (+1/-1; sign of v . o_C)
      counters     dict of diagnostics
    """

    def __init__(self, surface, N, ibcs=(), order=2, p=3, q=1, r=None,
                 tau_factor=0.1, check_factor=2.0, bc_types=None, band="tube"):
        if p not in (2, 3):
            raise ValueError("interpolation degree p must be 2 or 3")
        if band not in ("tube", "stencil_set"):
            raise ValueError("band is 'tube' or 'stencil_set'")
        self.band = band
        d = surface.dim
        self.surface, self.N, self.dim = surface, int(N), d
        self.p = int(p)
        self.h = 1.0 / N
        self.r = band_radius(N, d, p, q) if r is None else float(r)
        self.tau = tau_factor / float(N * N)
        self.inv_h2 = float(N) * float(N)
        self.order = int(order)
        K, CP = scan_band(surface, N, p, q, self.r)
        if band == "stencil_set":
            tube = CPMSystem(surface, N, ibcs, order, p, q, r, tau_factor, check_factor,
                             bc_types, band="tube")
            keep = stencil_set_nodes(tube)
            K, CP = K[keep], CP[keep]
        self.K, self.CP = K, CP
        self.n_s = n_s = K.shape[0]
        self.index = IndexMap(K)
        self.counters = dict(stencil_hole=0, no_bc_dof_swaps=0, on_c_nodes=0,
                             band_ties=int(np.sum(np.abs(
                                 np.sqrt(dot_rows(node_coords(K, N) - CP,
                                                  node_coords(K, N) - CP))
                                 - self.r) < 1e-12)))

        # ---- interior-boundary sets, BC DOF numbering (Sec. 4.1) ----
        self.sets = []
        bc_node, bc_curve = [], []
        alpha_of = []   # per C: (n_s,) BC DOF index or -1
        nxt = n_s
        for ci, curve in enumerate(ibcs):
            st = IBCSets(curve, K, CP, N, self.r, self.tau)
            # the check region scales with check_factor (paper: 2)
            if check_factor != 2.0:
                X = node_coords(K, N)
                D = X - curve.cp(X)
                st.in_check = np.sqrt(dot_rows(D, D)) < check_factor * self.r
                if hasattr(curve, "at_boundary"):
                    st.in_check &= ~curve.at_boundary(X)
            self.sets.append(st)
            amap = np.full(n_s, -1, dtype=np.int64)
            amap[st.omega_nodes] = nxt + np.arange(st.omega_nodes.size)
            nxt += st.omega_nodes.size
            alpha_of.append(amap)
            bc_node.append(st.omega_nodes)
            bc_curve.append(np.full(st.omega_nodes.size, ci))
            self.counters["on_c_nodes"] += int(st.on_c.sum())
        self.n_c = nxt - n_s
        self.n = nxt
        self.bc_node = np.concatenate(bc_node) if bc_node else np.zeros(0, np.int64)
        self.bc_curve = np.concatenate(bc_curve) if bc_curve else np.zeros(0, np.int64)
        self.alpha_of = alpha_of
        self.bc_cpc = (np.concatenate([s.cpc[s.omega_nodes] for s in self.sets])
                       if self.sets else np.zeros((0, d)))
        self.bc_side = (np.concatenate([s.side[s.omega_nodes] for s in self.sets])
                        if self.sets else np.zeros(0, np.int64))
        kinds = {"dirichlet": 0, "neumann": 1}
        if bc_types is None:
            bc_types = [("dirichlet", "dirichlet")] * len(ibcs)
        if len(bc_types) != len(ibcs):
            raise ValueError("one (side +1, side -1) condition pair per interior boundary")
        self.bc_types = [tuple(kinds[k] for k in pair) for pair in bc_types]
        # a BC DOF on side s serves side -s
        served = -self.bc_side
        self.bc_kind = np.array([self.bc_types[c][0 if sv > 0 else 1]
                                 for c, sv in zip(self.bc_curve, served)], dtype=np.int64)
        self.e_coef = np.where(self.bc_kind == 0, 2.0 if self.order == 2 else 1.0, 0.0)

        self._build_E()
        self._build_L()

    # ------------------------------------------------------------------
    def _members(self, base):
        offs = member_offsets(self.dim, self.p)
        MK = base[:, None, :] + offs[None, :, :]
        cols = self.index(MK)
        holes = int(np.sum(cols < 0))
        if holes:
            self.counters["stencil_hole"] += holes
            raise StencilHole("%d interpolation-stencil members are not band "
                              "nodes" % holes)
        return cols

    def _build_E(self):
        n_s, d = self.n_s, self.dim
        nm = (self.p + 1) ** d
        base, W = stencil(self.CP, self.N, d, self.p)
        cols0 = self._members(base)                     # (n_s, nm) PDE DOFs
        cols = cols0.copy()
        # PDE-row swaps (eq. stencil-crossing-test)
        for st, amap in zip(self.sets, self.alpha_of):
            rows = np.nonzero(st.in_check)[0]
            if rows.size == 0:
                continue
            C = cols0[rows]                             # (nr, nm)
            dot = dot_rows(st.v[rows][:, None, :], st.v[C])
            opp = dot < 0.0
            has_bc = amap[C] >= 0
            self.counters["no_bc_dof_swaps"] += int(np.sum(opp & ~has_bc & st.in_check[C]))
            swap = opp & has_bc
            if np.any(swap & (cols[rows] != C)):
                raise ValueError("two interior boundaries swap the same member")
            cols[rows] = np.where(swap, amap[C], cols[rows])
        r_idx = [np.repeat(np.arange(n_s), nm)]
        c_idx = [cols.ravel()]
        vals = [W.ravel()]
        # BC rows (Sec. 4.3): Dirichlet second order -w at cpbar_C; zero
        # Neumann +w at cp_C (first order) or cpbar_C (second order)
        for st, amap in zip(self.sets, self.alpha_of):
            nodes = st.omega_nodes
            if nodes.size == 0:
                continue
            kind = self.bc_kind[amap[nodes] - n_s]
            X = node_coords(self.K[nodes], self.N)
            Ybar = self.surface.cp(2.0 * st.cpc[nodes] - X)   # cpbar_C (eq. cpc-bar)
            if self.order == 2:
                Y, sign = Ybar, np.where(kind == 1, 1.0, -1.0)
                use = np.ones(nodes.size, dtype=bool)
            else:
                Y, sign = st.cpc[nodes], np.ones(nodes.size)
                use = kind == 1
            if not np.any(use):
                continue
            nodes, Y, sign = nodes[use], Y[use], sign[use]
            b2, W2 = stencil(Y, self.N, d, self.p)
            M = self._members(b2)
            dot = dot_rows(st.v[nodes][:, None, :], st.v[M])
            keep_bc = (dot >= 0.0) & (amap[M] >= 0)
            M2 = np.where(keep_bc, amap[M], M)
            r_idx.append(np.repeat(amap[nodes], nm))
            c_idx.append(M2.ravel())
            vals.append((sign[:, None] * W2).ravel())
        self.E = sp.csr_matrix((np.concatenate(vals),
                                (np.concatenate(r_idx), np.concatenate(c_idx))),
                               shape=(self.n, self.n))
        self.E.sum_duplicates()

    def _build_L(self):
        n_s, d = self.n_s, self.dim
        F = face_offsets(d)
        NB = self.index(self.K[:, None, :] + F[None, :, :])   # (n_s, 2d)
        present = NB >= 0
        cols0 = np.where(present, NB, 0)
        cols = cols0.copy()
        for st, amap in zip(self.sets, self.alpha_of):
            rows = np.nonzero(st.in_check)[0]
            if rows.size == 0:
                continue
            C = cols0[rows]
            P = present[rows]
            dot = dot_rows(st.v[rows][:, None, :], st.v[C])
            swap = (dot < 0.0) & (amap[C] >= 0) & P
            if np.any(swap & (cols[rows] != C)):
                raise ValueError("two interior boundaries swap the same neighbour")
            cols[rows] = np.where(swap, amap[C], cols[rows])
        rr = np.repeat(np.arange(n_s), 2 * d)[present.ravel()]
        cc = cols.ravel()[present.ravel()]
        r_idx, c_idx = [rr], [cc]
        # BC rows: neighbours restricted to Omega(C) (eq. FD-crossing-test);
        # past the end of an open curve the solution is single valued, so a
        # neighbour there without a BC DOF is its PDE DOF
        X = node_coords(self.K, self.N)
        for st, amap in zip(self.sets, self.alpha_of):
            nodes = st.omega_nodes
            if nodes.size == 0:
                continue
            past = (st.curve.at_boundary(X) if hasattr(st.curve, "at_boundary")
                    else np.zeros(n_s, dtype=bool))
            NBn = NB[nodes]
            ok = NBn >= 0
            NBc = np.where(ok, NBn, 0)
            has_bc = amap[NBc] >= 0
            ok &= has_bc | past[NBc]
            dot = dot_rows(st.v[nodes][:, None, :], st.v[NBc])
            col = np.where(has_bc, np.where(dot < 0.0, NBc, amap[NBc]), NBc)
            r_idx.append(np.repeat(amap[nodes], 2 * d)[ok.ravel()])
            c_idx.append(col.ravel()[ok.ravel()])
        r_idx = np.concatenate(r_idx)
        c_idx = np.concatenate(c_idx)
        off = sp.csr_matrix((np.full(r_idx.size, self.inv_h2), (r_idx, c_idx)),
                            shape=(self.n, self.n))
        off.sum_duplicates()
        self.L_off = off
        self.diagL = np.full(self.n, -2.0 * d * self.inv_h2)
        self.L = (off + sp.diags(self.diagL)).tocsr()

    # ------------------------------------------------------------------
    def apply(self, u, m, n):
        """The four-step matrix-vector product of Sec. 5.4 on the linear part:
        a = E u; b = (L - diag L) a; a = diag(L) u; v = m u + n a + n b."""
        a = self.E @ u
        b = self.L_off @ a
        a = self.diagL * u if u.ndim == 1 else self.diagL[:, None] * u
        return m * u + n * a + n * b

    def matrix(self, m, n):
        """Sparse A = m I + n [diag L + (L - diag L) E] (linear part)."""
        M = sp.diags(self.diagL) + self.L_off @ self.E
        return (m * sp.identity(self.n) + n * M).tocsr()

    def e_vector(self, g):
        """Constant part of the closest-point extension: zero on PDE DOFs,
        e_coef * g on BC DOFs."""
        e = np.zeros(self.n)
        e[self.n_s:] = self.e_coef * np.asarray(g, dtype=np.float64)
        return e

    def rhs(self, f_pde, g, n):
        """b = f - n (L - diag L) e(g), with f on BC DOFs copied from the PDE
        DOF of the same node (f is the closest-point extension of f-hat, which
        depends only on cp_S of the node)."""
        f = np.empty(self.n)
        f[:self.n_s] = f_pde
        f[self.n_s:] = np.asarray(f_pde)[self.bc_node]
        if self.n_c == 0:
            return f
        return f - n * (self.L_off @ self.e_vector(g))

    def surface_values(self, u, g=None):
        """E u + e at the PDE DOFs: the interpolated values at cp_S(x_i)."""
        e = self.e_vector(g) if (g is not None and self.n_c) else 0.0
        return (self.E @ u + e)[:self.n_s]

    # ------------------------------------------------------------------
    def row_of(self, i, m, n):
        """Row i of A as (columns, values), evaluated one entry at a time from
        E and L: used to check sampled outputs at sizes where the full product
        is not formed."""
        Erows = self.E
        Lrow = self.L_off.getrow(i)
        acc = {}
        acc[i] = m + n * self.diagL[i]
        for k, lk in zip(Lrow.indices, Lrow.data):
            er = Erows.getrow(k)
            for j, w in zip(er.indices, er.data):
                acc[j] = acc.get(j, 0.0) + n * lk * w
        cols = np.array(sorted(acc))
        return cols, np.array([acc[c] for c in cols])
