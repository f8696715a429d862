"""One whole ADER-MOOD step in 50-digit arithmetic (mpmath), for pinning
the FP64 oracle on tiny meshes.

TEST INFRASTRUCTURE.  Written from the paper and the readings the oracle
states, without the oracle's code: it imports nothing from ``oracle/`` or
from the HIP package.  It differs from the oracle in how it gets there:
  - corner vectors C_k = dV/dx_k from the derivative of the signed volume
    (eq. def_lcpncp), face measures and normals from them (|f_k| = d |C_k|,
    n_k = -C_k / |C_k|), so M_cp = z sum_{j != p} C_j C_j^T / |C_j| (R4);
  - derivatives of the stress (the chain rule of the predictor, R7) and of
    the pressure (the bulk modulus K_t of the sound speed, R5) by the
    complex step, T(tau + i h dtau, B + i h dB), h = 1e-40, exact far
    below FP64 roundoff;
  - the least-squares fit (R8), the nodal systems (R14, R22) and the
    Crank-Nicolson B update (R10) as mpmath linear solves.
The cascade is the two-level one (R18): flagged cells go to first order
and the step is recomputed from t^n until no new cell is flagged.
Neo-Hookean law only (eq. cstnh with K = lambda + 2 mu / 3, R1).
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 50
_H = mp.mpf("1e-40")


def _f(x):
    return mp.mpf(float(x))


def _z3():
    return [[mp.mpf(0)] * 3 for _ in range(3)]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _bad(v):
    return mp.isnan(v) or mp.isinf(v)


def _solve(A, b):
    """Solve the small dense system A x = b (lists) in mpmath; a system
    holding a non-finite value gives NaNs, as FP64 elimination would."""
    if any(_bad(v) for row in A for v in row) or any(_bad(v) for v in b):
        return [mp.nan] * len(b)
    return list(mp.lu_solve(mp.matrix(A), mp.matrix(b)))


def _ln(x):
    """log with IEEE semantics on the reals: NaN for x <= 0 (the complex
    step passes x with a tiny imaginary part and a positive real part)."""
    re = mp.re(x) if isinstance(x, mp.mpc) else x
    if _bad(re) or not re > 0:
        return mp.nan
    return mp.log(x)


def _sqrt(x):
    if _bad(x) or not x >= 0:
        return mp.nan
    return mp.sqrt(x)


# ------------------------------------------------------------ geometry
def geometry(d, X):
    """X: d+1 points as 3-lists (third component 0 in 2D).  Returns the
    signed measure V, the corner vectors C[k] = dV/dx_k (3-lists), their
    norms, the centroid and the in-sphere diameter 2 d V / sum |f|."""
    if d == 3:
        e1, e2, e3 = ([X[k][i] - X[0][i] for i in range(3)] for k in (1, 2, 3))
        C1 = [v / 6 for v in _cross(e2, e3)]
        C2 = [v / 6 for v in _cross(e3, e1)]
        C3 = [v / 6 for v in _cross(e1, e2)]
        V = _dot(e1, C1)
        C = [[-(C1[i] + C2[i] + C3[i]) for i in range(3)], C1, C2, C3]
    else:
        e1 = [X[1][i] - X[0][i] for i in range(2)]
        e2 = [X[2][i] - X[0][i] for i in range(2)]
        V = (e1[0] * e2[1] - e1[1] * e2[0]) / 2
        C1 = [e2[1] / 2, -e2[0] / 2, mp.mpf(0)]
        C2 = [-e1[1] / 2, e1[0] / 2, mp.mpf(0)]
        C = [[-(C1[i] + C2[i]) for i in range(3)], C1, C2]
    cn = [mp.sqrt(_dot(c, c)) for c in C]
    xc = [sum(X[k][i] for k in range(d + 1)) / (d + 1) for i in range(3)]
    faces = sum(d * n for n in cn)       # |f_k| = d |C_k|
    return dict(V=V, C=C, cn=cn, xc=xc, Lc=2 * d * V / faces)


def corner_shape(g, p, nv):
    """sum over the faces of c through p of (|f|/d) n_f n_f^T."""
    N = _z3()
    for j in range(nv):
        if j == p:
            continue
        Cj, r = g["C"][j], g["cn"][j]
        for a in range(3):
            for b in range(3):
                N[a][b] += Cj[a] * Cj[b] / r
    return N


# ---------------------------------------------------- constitutive law
def pressure(K, J):
    return -(K / 2) * (J - 1 + _ln(J) / J)


def stress(rho0, mu, K, tau, B):
    """T = -p I + mu J^(-5/3) dev B, J = rho0 tau (eq. cstnh, R1, R2); real
    or complex arguments."""
    J = rho0 * tau
    p = pressure(K, J)
    f = mp.exp(-mp.mpf(5) / 3 * _ln(J))
    t = (B[0][0] + B[1][1] + B[2][2]) / 3
    return [[mu * f * (B[i][j] - (t if i == j else 0)) - (p if i == j else 0) for j in range(3)] for i in range(3)]


def stress_derivative(rho0, mu, K, tau, B, dtau, dB):
    Tc = stress(rho0, mu, K, mp.mpc(tau, _H * dtau),
                [[mp.mpc(B[i][j], _H * dB[i][j]) for j in range(3)] for i in range(3)])
    return [[mp.im(Tc[i][j]) / _H for j in range(3)] for i in range(3)]


def sound_speed(rho0, mu, K, tau):
    """a^2 = tau (K_t + 4 mu / 3) with K_t = -J dp/dJ (R5)."""
    J = rho0 * tau
    dpdJ = mp.im(pressure(K, mp.mpc(J, _H))) / _H
    return _sqrt(tau * (-J * dpdJ + 4 * mu / 3))


def free_energy(rho0, mu, K, tau, B):
    J = rho0 * tau
    I1b = (B[0][0] + B[1][1] + B[2][2]) * mp.exp(-mp.mpf(2) / 3 * _ln(J))
    return K / (4 * rho0) * ((J - 1) ** 2 + _ln(J) ** 2) + mu / (2 * rho0) * (I1b - 3)


def _det3(A):
    return mp.det(mp.matrix(A))


# ------------------------------------------------------------ the step
class MPProblem:
    """Mesh, walls and material in 50-digit arithmetic.  Arrays are plain
    lists or numpy arrays of doubles in the C-ABI layout."""

    def __init__(self, dim, x0, cells, nwall, normals, rho0, mu, lam):
        self.d = d = int(dim)
        self.nv = d + 1
        self.cells = [[int(p) for p in c] for c in cells]
        self.nn = len(x0)
        self.nc = len(self.cells)
        self.rho0 = [_f(r) for r in rho0]
        self.mu = [_f(m) for m in mu]
        self.K = [_f(l) + 2 * _f(m) / 3 for l, m in zip(lam, mu)]
        self.node_cells = [[] for _ in range(self.nn)]
        for c, nodes in enumerate(self.cells):
            for k, p in enumerate(nodes):
                self.node_cells[p].append((c, k))
        X0 = [self._pt(x0[p]) for p in range(self.nn)]
        self.m = [self.rho0[c] * geometry(d, [X0[p] for p in self.cells[c]])["V"] for c in range(self.nc)]
        # orthonormal basis of the allowed directions of every node
        self.basis = []
        for p in range(self.nn):
            Q = []
            for r in range(int(nwall[p])):
                w = [_f(normals[p][r][i]) for i in range(d)]
                for q in Q:
                    s = sum(w[i] * q[i] for i in range(d))
                    w = [w[i] - s * q[i] for i in range(d)]
                n = mp.sqrt(sum(v * v for v in w))
                if n > mp.mpf("1e-8"):
                    Q.append([v / n for v in w])
            P = []
            for a in range(d):
                if len(Q) + len(P) == d:
                    break
                w = [mp.mpf(1) if i == a else mp.mpf(0) for i in range(d)]
                for q in Q + P:
                    s = sum(w[i] * q[i] for i in range(d))
                    w = [w[i] - s * q[i] for i in range(d)]
                n = mp.sqrt(sum(v * v for v in w))
                if n > mp.mpf("1e-8"):
                    P.append([v / n for v in w])
            self.basis.append(P)

    def _pt(self, x):
        return [_f(x[i]) if i < self.d else mp.mpf(0) for i in range(3)]

    def _B(self, b):
        b = [_f(v) for v in b]
        if self.d == 3:
            return [[b[0], b[3], b[4]], [b[3], b[1], b[5]], [b[4], b[5], b[2]]]
        return [[b[0], b[2], mp.mpf(0)], [b[2], b[1], mp.mpf(0)], [mp.mpf(0), mp.mpf(0), mp.mpf(1)]]

    def _sym(self):
        return [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)] if self.d == 3 else [(0, 0), (1, 1), (0, 1)]

    def step(self, state, dt, params, mask=None, detect=True):
        """One step from ``state`` (dict of x, vhat, tau, v, e, B arrays).
        params: dict of c_cfl, c_v, c_i, delta0, delta1, eps_tol.  mask:
        cells forced to first order; detect False takes the mask as given.
        Returns (new state, vstar, mask, info), values as mpf."""
        d, nv, nc, nn = self.d, self.nv, self.nc, self.nn
        dt = _f(dt)
        x = [self._pt(state["x"][p]) for p in range(nn)]
        vh = [self._pt(state["vhat"][p]) for p in range(nn)]
        tau = [_f(t) for t in state["tau"]]
        v = [self._pt(state["v"][c]) for c in range(nc)]
        e = [_f(t) for t in state["e"]]
        B = [self._B(state["B"][c]) for c in range(nc)]
        geo = [geometry(d, [x[p] for p in self.cells[c]]) for c in range(nc)]
        grads = self._lsq(geo, tau, v, B)
        # relaxed-DMP bounds of rho^n (eq. RDMP, R17): {c} and its stencil
        rlo, rhi = [], []
        for c in range(nc):
            rs = [1 / tau[j] for p in self.cells[c] for (j, _) in self.node_cells[p]] + [1 / tau[c]]
            rlo.append(min(rs))
            rhi.append(max(rs))
        mk = [0] * nc if mask is None else [int(k) for k in mask]
        iters, first = 0, None
        while True:
            out = self._candidate(geo, grads, x, vh, tau, v, e, B, dt, mk)
            iters += 1
            if not detect:
                first = 0
                break
            flags = []
            for c in range(nc):
                if mk[c] >= 2:
                    continue
                if self._inadmissible(out, c, params) or self._rdmp(out, c, rlo[c], rhi[c], params):
                    flags.append(c)
            if first is None:
                first = len(flags)
            if not flags:
                break
            for c in flags:
                mk[c] = 2
        x1, vh1, tau1, v1, e1, B1, vs = out
        info = dict(mood_iters=iters, n_flag_first=first, n_p0=sum(1 for k in mk if k == 2))
        info.update(self._dt(x1, tau1, tau, dt, params))
        info.update(self._diag(tau1, v1, e1, B1))
        new = dict(x=x1, vhat=vh1, tau=tau1, v=v1, e=e1, B=B1)
        return new, vs, mk, info

    # ---------------------------------------------------- reconstruction
    def _W(self, tau, v, B, c):
        return [tau[c]] + [v[c][i] for i in range(self.d)] + [B[c][i][j] for (i, j) in self._sym()]

    def _lsq(self, geo, tau, v, B):
        """Unweighted least squares over every cell sharing a node with c,
        one visit per shared node (R8); a stencil that cannot fix a gradient
        (fewer than d visits, or a singular normal matrix) gives zero."""
        d = self.d
        out = []
        for c in range(self.nc):
            Wc = self._W(tau, v, B, c)
            nW = len(Wc)
            A = [[mp.mpf(0)] * d for _ in range(d)]
            b = [[mp.mpf(0)] * d for _ in range(nW)]
            visits = 0
            for p in self.cells[c]:
                for (j, _) in self.node_cells[p]:
                    if j == c:
                        continue
                    visits += 1
                    dx = [geo[j]["xc"][i] - geo[c]["xc"][i] for i in range(d)]
                    Wj = self._W(tau, v, B, j)
                    for a in range(d):
                        for q in range(d):
                            A[a][q] += dx[a] * dx[q]
                    for w in range(nW):
                        for a in range(d):
                            b[w][a] += dx[a] * (Wj[w] - Wc[w])
            tr = sum(A[a][a] for a in range(d))
            det = mp.det(mp.matrix(A))
            if visits < d or not tr > 0 or not det > mp.mpf("1e-12") * (tr / d) ** d:
                out.append([[mp.mpf(0)] * d for _ in range(nW)])
                continue
            out.append([_solve(A, b[w]) for w in range(nW)])
        return out

    # -------------------------------------------------------- candidate
    def _candidate(self, geo, grads, x, vh, tau, v, e, B, dt, mk):
        d, nv, nc, nn = self.d, self.nv, self.nc, self.nn
        sym = self._sym()
        h = dt / 2
        cor = {}
        for c in range(nc):
            rho0, mu, K = self.rho0[c], self.mu[c], self.K[c]
            g = grads[c]
            G = _z3()
            dT = [None] * d
            if mk[c] < 2:
                for i in range(d):
                    for j in range(d):
                        G[i][j] = g[1 + i][j]
                for j in range(d):
                    dB = _z3()
                    for s, (a, b) in enumerate(sym):
                        dB[a][b] = dB[b][a] = g[1 + d + s][j]
                    dT[j] = (g[0][j], dB)
            if mk[c] < 2:
                # time derivatives at the cell centre (R7): tau tr G, tau div T
                # (chain rule through T(tau, B)), G B + B G^T
                trG = sum(G[i][i] for i in range(3))
                divT = [mp.mpf(0)] * 3
                for j in range(d):
                    D = stress_derivative(rho0, mu, K, tau[c], B[c], dT[j][0], dT[j][1])
                    for i in range(3):
                        divT[i] += D[i][j]
                GB = [[sum(G[i][q] * B[c][q][j] + B[c][i][q] * G[j][q] for q in range(3)) for j in range(3)]
                      for i in range(3)]
            for k, p in enumerate(self.cells[c]):
                if mk[c] >= 2:
                    ts, vs, Bs = tau[c], v[c][:], [row[:] for row in B[c]]
                else:
                    delta = [x[p][i] - geo[c]["xc"][i] for i in range(3)]
                    ts = tau[c] + sum(g[0][j] * delta[j] for j in range(d)) + h * tau[c] * trG
                    vs = [v[c][i] + sum(G[i][j] * delta[j] for j in range(d)) + h * tau[c] * divT[i]
                          if i < d else mp.mpf(0) for i in range(3)]
                    Bs = [row[:] for row in B[c]]
                    for s, (a, b) in enumerate(sym):
                        val = B[c][a][b] + sum(dT[j][1][a][b] * delta[j] for j in range(d)) + h * GB[a][b]
                        Bs[a][b] = Bs[b][a] = val
                T = stress(rho0, mu, K, ts, Bs)
                z = sound_speed(rho0, mu, K, ts) / ts
                cor[(c, k)] = (vs, T, z, corner_shape(geo[c], k, nv))
        # nodal solver (R14, R15, R22)
        vstar = []
        for p in range(nn):
            M = _z3()
            r = [mp.mpf(0)] * 3
            for (c, k) in self.node_cells[p]:
                vs, T, z, N = cor[(c, k)]
                Cc = geo[c]["C"][k]
                for a in range(3):
                    for b in range(3):
                        M[a][b] += z * N[a][b]
                    r[a] += sum(z * N[a][b] * vs[b] - T[a][b] * Cc[b] for b in range(3))
            P = self.basis[p]
            m = len(P)
            if not self.node_cells[p] or m == 0:
                vstar.append([mp.mpf(0)] * 3)
                continue
            A = [[sum(P[s][i] * M[i][j] * P[t][j] for i in range(d) for j in range(d)) for t in range(m)]
                 for s in range(m)]
            rhs = [sum(P[s][i] * r[i] for i in range(d)) for s in range(m)]
            al = _solve(A, rhs)
            vstar.append([sum(P[t][i] * al[t] for t in range(m)) if i < d else mp.mpf(0) for i in range(3)])
        x1 = [[x[p][i] + dt * vstar[p][i] if i < d else mp.mpf(0) for i in range(3)] for p in range(nn)]
        vh1 = [[2 * vstar[p][i] - vh[p][i] for i in range(3)] for p in range(nn)]
        # cell update (R12, R13, R15) and B (R10, R11)
        tau1, v1, e1, B1 = [], [], [], []
        for c in range(nc):
            g0 = geo[c]
            F = [mp.mpf(0)] * 3
            W = mp.mpf(0)
            for k, p in enumerate(self.cells[c]):
                vs, T, z, N = cor[(c, k)]
                f = [sum(T[a][b] * g0["C"][k][b] + z * N[a][b] * (vstar[p][b] - vs[b]) for b in range(3))
                     for a in range(3)]
                for a in range(3):
                    F[a] += f[a]
                W += _dot(f, vstar[p])
            mc = self.m[c]
            v1.append([v[c][i] + dt / mc * F[i] for i in range(3)])
            e1.append(e[c] + dt / mc * W)
            g1 = geometry(d, [x1[p] for p in self.cells[c]])
            tau1.append(g1["V"] / mc)
            if mk[c] < 2:
                L0 = self._L(g0, [vh[p] for p in self.cells[c]])
                L1 = self._L(g1, [vh1[p] for p in self.cells[c]])
                B1.append(self._cn(B[c], L0, L1, dt))
            else:
                L = self._L(g0, [vstar[p] for p in self.cells[c]])
                Y = [[sum(L[i][q] * B[c][q][j] + B[c][i][q] * L[j][q] for q in range(3)) for j in range(3)]
                     for i in range(3)]
                Bn = [[B[c][i][j] + dt * Y[i][j] for j in range(3)] for i in range(3)]
                if d == 2:
                    Bn[2][2] = mp.mpf(1)
                B1.append(Bn)
        return x1, vh1, tau1, v1, e1, B1, vstar

    def _L(self, g, vp):
        """L = (1/V) sum_p v_p (x) C_p (R6)."""
        return [[sum(vp[k][i] * g["C"][k][j] for k in range(self.nv)) / g["V"] for j in range(3)] for i in range(3)]

    def _cn(self, Bn, L0, L1, dt):
        """Crank-Nicolson: X - (dt/2)(L1 X + X L1^T) = Bn + (dt/2)(L0 Bn + Bn L0^T)
        for the symmetric X (R10)."""
        sym = self._sym()
        Y = [[sum(L0[i][q] * Bn[q][j] + Bn[i][q] * L0[j][q] for q in range(3)) for j in range(3)] for i in range(3)]
        rhs = [Bn[a][b] + dt / 2 * Y[a][b] for (a, b) in sym]
        A = [[mp.mpf(0)] * len(sym) for _ in sym]
        for col, (a, b) in enumerate(sym):
            E = _z3()
            E[a][b] = E[b][a] = mp.mpf(1)
            Z = [[sum(L1[i][q] * E[q][j] + E[i][q] * L1[j][q] for q in range(3)) for j in range(3)] for i in range(3)]
            for row, (i, j) in enumerate(sym):
                A[row][col] = E[i][j] - dt / 2 * Z[i][j]
        s = _solve(A, rhs)
        X = _z3()
        for q, (a, b) in enumerate(sym):
            X[a][b] = X[b][a] = s[q]
        if self.d == 2:
            X[2][2] = mp.mpf(1)
        return X

    # --------------------------------------------------------- detection
    def _inadmissible(self, out, c, prm):
        """eq. PAD with R16: finite, tau > 0, det B > 0, eps >= -tol (|e| +
        |v|^2/2)."""
        _, _, tau1, v1, e1, B1, _ = out
        vals = [tau1[c], e1[c]] + list(v1[c]) + [b for row in B1[c] for b in row]
        if any(_bad(v) for v in vals):
            return True
        if not tau1[c] > 0:
            return True
        if not _det3(B1[c]) > 0:
            return True
        k2 = _dot(v1[c], v1[c])
        eps = e1[c] - k2 / 2
        return eps < -_f(prm["eps_tol"]) * (abs(e1[c]) + k2 / 2)

    def _rdmp(self, out, c, lo, hi, prm):
        rho1 = 1 / out[2][c]
        delta = max(_f(prm["delta0"]), _f(prm["delta1"]) * (hi - lo))
        return rho1 < lo - delta or rho1 > hi + delta

    # ------------------------------------------------------- time step
    def _dt(self, x1, tau1, tau0, dt, prm):
        """eqs. CFL, CFL2 with R20, R21."""
        ac = None
        vol = None
        for c in range(self.nc):
            g = geometry(self.d, [x1[p] for p in self.cells[c]])
            r = g["Lc"] / sound_speed(self.rho0[c], self.mu[c], self.K[c], tau1[c])
            ac = r if ac is None else min(ac, r)
            V1, V0 = self.m[c] * tau1[c], self.m[c] * tau0[c]
            if V1 != V0:
                q = V1 / abs(V1 - V0)
                vol = q if vol is None else min(vol, q)
        out = dict(dt_acoustic=_f(prm["c_cfl"]) * ac)
        dtp = dt
        if dtp > 0:
            out["dt_volume"] = _f(prm["c_v"]) * dtp * vol if vol is not None else mp.inf
            out["dt_next"] = min(out["dt_acoustic"], out["dt_volume"], (1 + _f(prm["c_i"])) * dtp)
        else:
            out["dt_volume"] = mp.inf
            out["dt_next"] = out["dt_acoustic"]
        return out

    def _diag(self, tau1, v1, e1, B1):
        m = self.m
        return dict(mass=sum(m), mom=[sum(m[c] * v1[c][i] for c in range(self.nc)) for i in range(3)],
                    energy=sum(m[c] * e1[c] for c in range(self.nc)),
                    kinetic=sum(m[c] * _dot(v1[c], v1[c]) / 2 for c in range(self.nc)),
                    elastic=sum(m[c] * free_energy(self.rho0[c], self.mu[c], self.K[c], tau1[c], B1[c])
                                for c in range(self.nc)))

    def pack(self, st):
        """Convert a step's output to double arrays in the C-ABI layout."""
        import numpy as np
        d = self.d
        sym = self._sym()
        return dict(x=np.array([[float(p[i]) for i in range(d)] for p in st["x"]]),
                    vhat=np.array([[float(p[i]) for i in range(d)] for p in st["vhat"]]),
                    tau=np.array([float(t) for t in st["tau"]]),
                    v=np.array([[float(p[i]) for i in range(d)] for p in st["v"]]),
                    e=np.array([float(t) for t in st["e"]]),
                    B=np.array([[float(b[i][j]) for (i, j) in sym] for b in st["B"]]))
