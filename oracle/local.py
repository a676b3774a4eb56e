"""Row-by-row evaluation of (A u) at sampled nodes, for checks at grid sizes
where the full system (explicit E and L) is too large to assemble.

The definitions are those of ``operator.CPMSystem`` (Sec. 3.2, 4.3, 5.3,
5.4), evaluated only for the requested rows:

    (A u)_i = (m + n D) u_i + n N^2 sum_{k in FD(i)} (E u)_{col(k)}

where col(k) is the FD column of row i after the crossing test (eq.
stencil-crossing-test for PDE rows, eq. FD-crossing-test for BC rows) and
(E u)_c the interpolation row of column c: the stencil of cp_S with swaps
for a PDE column, the second-order mirror stencil (eq. cpc-bar) for a BC
column.  Every node property (band membership, cp_S, cp_C, side vector,
Omega(C), check region) is recomputed from its definition at the node.

Values u are supplied through a callback u_of(K, curve) -> array, where K
holds integer node coordinates and curve is -1 for PDE DOFs and the index of
the interior boundary for BC DOFs.  This module is test infrastructure; it is
pinned against ``CPMSystem.apply`` in ``tests/test_oracle_local.py``.

Scope: the full tube (eq. bandwidth), cubic interpolation (p = 3), closed
interior boundaries (points, closed curves) with Dirichlet conditions of
order 1 (the BC row's linear part is zero, Sec. 4.3) or 2 (the mirror row of
eq. cpc-bar).  Anything else - zero-Neumann sides, open arcs (whose end
nodes have no BC DOF, Sec. 4.4), quadratic interpolation, the stencil-set
band - is refused with NotImplementedError rather than evaluated with the
rules above.
"""

import numpy as np

from .band import band_radius, dot_rows, node_coords
from .operator import face_offsets, member_offsets, stencil


class LocalCPM:
    def __init__(self, surface, N, curves=(), order=2, tau_factor=0.1, check_factor=2.0,
                 bc_types=None, p=3, band="tube"):
        from .geometry import LatitudeArc
        if int(order) not in (1, 2):
            raise NotImplementedError("IBC order %r: only orders 1 and 2 exist (Sec. 4.3)" % order)
        if p != 3:
            raise NotImplementedError("the row evaluator models cubic interpolation only")
        if band != "tube":
            raise NotImplementedError("the row evaluator models the full tube only")
        if bc_types is not None and any(t != "dirichlet" for pair in bc_types for t in pair):
            raise NotImplementedError("the row evaluator models Dirichlet interior boundaries only")
        if any(isinstance(C, LatitudeArc) for C in curves):
            raise NotImplementedError("the row evaluator models closed interior boundaries only")
        self.S, self.N, self.dim = surface, int(N), surface.dim
        self.curves = list(curves)
        self.order = int(order)
        self.r = band_radius(N, self.dim)
        self.tau = tau_factor / float(N * N)
        self.cf = check_factor
        self.inv_h2 = float(N) * float(N)

    # --------------------------------------------------------- node props
    def _props(self, K):
        """cp_S, band flag, and per curve (cp_C, d_C, side vector)."""
        X = node_coords(K, self.N)
        CP = self.S.cp(X)
        D = X - CP
        inb = np.sqrt(dot_rows(D, D)) <= self.r
        per = []
        for C in self.curves:
            CPC = C.cp(X)
            E = X - CPC
            dC = np.sqrt(dot_rows(E, E))
            V = CP - CPC
            nv = np.sqrt(dot_rows(V, V))
            on = nv < self.tau
            O = C.orient(CPC)
            V[on] = self.tau * O[on]
            per.append((CPC, dC, V))
        return X, CP, inb, per

    def _curve_of(self, per):
        """Index of the curve whose check region holds the node (or -1)."""
        n = per[0][1].shape[0] if per else 0
        c = np.full(n, -1)
        for ci, (_, dC, _) in enumerate(per):
            c = np.where((c < 0) & (dC < self.cf * self.r), ci, c)
        return c

    # ------------------------------------------------------- E rows
    def _E_pde(self, K, u_of):
        """(E u) at PDE nodes K (all in the band)."""
        s, d = K.shape
        _, CP, _, per = self._props(K)
        base, W = stencil(CP, self.N, d)
        offs = member_offsets(d)
        MK = (base[:, None, :] + offs[None, :, :]).reshape(-1, d)
        _, _, minb, mper = self._props(MK)
        assert np.all(minb), "stencil hole"
        curve = np.full(MK.shape[0], -1)
        if self.curves:
            rc = self._curve_of(per)
            for ci, ((_, dC, V), (_, mdC, mV)) in enumerate(zip(per, mper)):
                rows = np.repeat(rc == ci, offs.shape[0])
                vi = np.repeat(V, offs.shape[0], axis=0)
                swap = rows & (mdC <= self.r) & (dot_rows(vi, mV) < 0.0)
                curve = np.where(swap, ci, curve)
        vals = u_of(MK, curve).reshape(s, -1)
        return np.sum(W * vals, axis=1)

    def _E_bc(self, K, ci, u_of):
        """(E u) at the BC DOFs of curve ci at nodes K (linear part): zero for
        a first-order Dirichlet row (its value is the constant g), minus the
        mirror-point interpolation for a second-order one."""
        s, d = K.shape
        if self.order == 1:
            return np.zeros(s)
        X, _, _, per = self._props(K)
        CPC, _, V = per[ci]
        Y = self.S.cp(2.0 * CPC - X)
        base, W = stencil(Y, self.N, d)
        offs = member_offsets(d)
        MK = (base[:, None, :] + offs[None, :, :]).reshape(-1, d)
        _, _, minb, mper = self._props(MK)
        assert np.all(minb), "mirror stencil hole"
        _, mdC, mV = mper[ci]
        vj = np.repeat(V, offs.shape[0], axis=0)
        keep_bc = (mdC <= self.r) & ~(dot_rows(vj, mV) < 0.0)
        curve = np.where(keep_bc, ci, -1)
        vals = u_of(MK, curve).reshape(s, -1)
        return -np.sum(W * vals, axis=1)

    def _E_cols(self, K, curve, u_of):
        out = np.zeros(K.shape[0])
        m = curve < 0
        if m.any():
            out[m] = self._E_pde(K[m], u_of)
        for ci in range(len(self.curves)):
            mm = curve == ci
            if mm.any():
                out[mm] = self._E_bc(K[mm], ci, u_of)
        return out

    # ------------------------------------------------------- A rows
    def apply_rows(self, K, curve, u_of, m, n):
        """(A u) for sampled DOFs: node coordinates K (s, d) and curve (s,)
        (-1 for a PDE DOF, else the interior boundary of the BC DOF)."""
        K = np.asarray(K, dtype=np.int64)
        curve = np.asarray(curve)
        s, d = K.shape
        F = face_offsets(d)
        NK = (K[:, None, :] + F[None, :, :]).reshape(-1, d)
        _, _, ninb, nper = self._props(NK)
        _, _, _, per = self._props(K)
        rowc = np.repeat(curve, F.shape[0])
        ncurve = np.full(NK.shape[0], -1)
        present = ninb.copy()
        if self.curves:
            rc = np.repeat(self._curve_of(per), F.shape[0])
            for ci, ((_, _, V), (_, ndC, nV)) in enumerate(zip(per, nper)):
                vi = np.repeat(V, F.shape[0], axis=0)
                opp = dot_rows(vi, nV) < 0.0
                in_om = (ndC <= self.r) & ninb
                # PDE rows in the check region: swap opposite-side neighbours
                ncurve = np.where((rowc < 0) & (rc == ci) & in_om & opp, ci, ncurve)
                # BC rows: only neighbours in Omega(C); same side stays BC
                bc = rowc == ci
                present = np.where(bc, in_om, present)
                ncurve = np.where(bc & in_om & ~opp, ci, ncurve)
        Eu = np.zeros(NK.shape[0])
        if present.any():
            Eu[present] = self._E_cols(NK[present], ncurve[present], u_of)
        off = np.sum(Eu.reshape(s, -1), axis=1)
        ui = u_of(K, curve)
        D = -2.0 * d * self.inv_h2
        return (m + n * D) * ui + n * self.inv_h2 * off
