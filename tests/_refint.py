"""Independent high-accuracy reference for one element pair (test helper).

Computes L_ab = int_{T_k} int_{T_l} Psi(x - y) a_a a_b dy dx with
a = phi(x) - phi(y) over the union nodes of T_k and T_l, for kernels of the
form Psi(z) = c |z|^-alpha K(z/|z|) (constant: alpha = 0, K = 1;
1/|z|: alpha = 1, K = 1; peridynamic: alpha = 1, K = e e^T).

Route (no regularising transforms of T x T, nothing shared with the oracle):
* the inner integral over T_l at a fixed outer point x is split into the
  signed triangles (x, a, b) over the edges (a, b) of T_l; each is mapped by
  y = x + t (a - x + s (b - a)), dy = t |det(a - x, b - a)| ds dt, so the
  t-integral of (polynomial in t) * t^(1 - alpha) is exact in closed form;
* the remaining s-integral carries |a - x + s (b - a)|^-alpha, nearly
  singular when x is close to the line ab; it is taken with the sinh
  transformation of Johnston and Elliott (s = s0 + (d/L) sinh u around the
  foot point s0 of x) and 40-point Gauss-Legendre pieces;
* the outer integral over T_k uses scipy's adaptive ``quad_vec`` twice
  (reference coordinates xi_1, then xi_2).
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad_vec

_GX, _GW = np.polynomial.legendre.leggauss(40)


def _basis_grad(V):
    """Gradients of the three P1 basis functions of triangle V (3x2) and
    their values' affine form: phi_a(y) = g_a . (y - V0) + phi_a(V0)."""
    J = np.array([V[1] - V[0], V[2] - V[0]]).T       # columns v1-v0, v2-v0
    Jinv = np.linalg.inv(J)
    # phi_1 = xi_1, phi_2 = xi_2, phi_0 = 1 - xi_1 - xi_2 ; xi = Jinv (y - V0)
    g1, g2 = Jinv[0], Jinv[1]
    return np.array([-(g1 + g2), g1, g2])


def _phi(V, G, y):
    """Basis values of triangle V at points y (..., 2) -> (..., 3)."""
    d = y - V[0]
    p1 = d @ G[1]
    p2 = d @ G[2]
    return np.stack([1.0 - p1 - p2, p1, p2], axis=-1)


def _halfplanes(V):
    """Outward normals n_i and offsets c_i with T = {n_i . y <= c_i}."""
    orient = np.sign((V[1, 0] - V[0, 0]) * (V[2, 1] - V[0, 1]) -
                     (V[1, 1] - V[0, 1]) * (V[2, 0] - V[0, 0]))
    ns, cs = [], []
    for i in range(3):
        a, b = V[i], V[(i + 1) % 3]
        e = b - a
        n = orient * np.array([e[1], -e[0]])
        ns.append(n)
        cs.append(n @ a)
    return np.array(ns), np.array(cs)


class PairIntegral:
    def __init__(self, Vk, Vl, nodes_k, nodes_l, kernel, c):
        self.Vk = np.asarray(Vk, float)
        self.Vl = np.asarray(Vl, float)
        self.Gk = _basis_grad(self.Vk)
        self.Gl = _basis_grad(self.Vl)
        self.Nl, self.Cl = _halfplanes(self.Vl)
        d = self.Vl[1:] - self.Vl[0]
        self.orient_l = np.sign(d[0, 0] * d[1, 1] - d[0, 1] * d[1, 0])
        union = list(nodes_k)
        for b in nodes_l:
            if b not in union:
                union.append(b)
        self.union = union
        self.ink = [list(nodes_k).index(u) if u in nodes_k else -1 for u in union]
        self.inl = [list(nodes_l).index(u) if u in nodes_l else -1 for u in union]
        self.kernel = kernel
        self.c = c
        self.alpha = 0.0 if kernel == "constant" else 1.0
        self.ncomp = 2 if kernel == "peridynamic" else 1

    def _edge_nodes(self, x, a, b):
        """s-nodes and weights on [0, 1] for the segment a -> b seen from x."""
        ab = b - a
        L2 = ab @ ab
        s0 = (x - a) @ ab / L2
        foot = a + s0 * ab
        eta = np.sqrt(max((x - foot) @ (x - foot), 0.0) / L2)
        if eta > 0.25:
            return 0.5 * (_GX + 1.0), 0.5 * _GW
        eta = max(eta, 1e-300)
        ss, ws = [], []
        cuts = [0.0, 1.0] if (s0 <= 0.0 or s0 >= 1.0) else [0.0, s0, 1.0]
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            u0 = np.arcsinh((lo - s0) / eta)
            u1 = np.arcsinh((hi - s0) / eta)
            # split long u-ranges geometrically so every piece stays smooth
            nseg = max(1, int(np.ceil(abs(u1 - u0) / 2.0)))
            edges = np.linspace(u0, u1, nseg + 1)
            for p, q in zip(edges[:-1], edges[1:]):
                u = 0.5 * (q - p) * _GX + 0.5 * (q + p)
                wu = 0.5 * (q - p) * _GW
                ss.append(s0 + eta * np.sinh(u))
                ws.append(wu * eta * np.cosh(u))
        return np.concatenate(ss), np.concatenate(ws)

    def inner(self, x):
        """Matrix-valued inner integral at the outer point x."""
        pk = _phi(self.Vk, self.Gk, x)      # basis of T_k at x
        pl = _phi(self.Vl, self.Gl, x)      # affine extension of T_l's basis at x
        nu = len(self.union)
        A = np.zeros(nu)
        Gr = np.zeros((nu, 2))
        for u in range(nu):
            fx = pk[self.ink[u]] if self.ink[u] >= 0 else 0.0
            py = pl[self.inl[u]] if self.inl[u] >= 0 else 0.0
            A[u] = fx - py
            if self.inl[u] >= 0:
                Gr[u] = self.Gl[self.inl[u]]
        al = self.alpha
        c0, c1, c2 = 1.0 / (2.0 - al), 1.0 / (3.0 - al), 1.0 / (4.0 - al)
        n = self.ncomp
        out = np.zeros((nu, n, nu, n))
        for i in range(3):
            a, b = self.Vl[i], self.Vl[(i + 1) % 3]
            det = (a[0] - x[0]) * (b[1] - a[1]) - (a[1] - x[1]) * (b[0] - a[0])
            if det == 0.0:
                continue
            s, ws = self._edge_nodes(x, a, b)
            w = (a - x)[None, :] + s[:, None] * (b - a)[None, :]      # (S, 2)
            rw = np.sqrt(np.sum(w * w, axis=1))
            Dw = w @ Gr.T                                              # (S, nu)
            base = ws * (det * self.orient_l) * rw ** (-al)            # signed
            for cc in range(n):
                for dd in range(n):
                    if n == 1:
                        kw = base
                    else:
                        kw = base * w[:, cc] * w[:, dd] / (rw * rw)
                    S0 = np.sum(kw)
                    S1 = kw @ Dw
                    S2 = (Dw * kw[:, None]).T @ Dw
                    out[:, cc, :, dd] += (np.outer(A, A) * S0 * c0
                                          - (np.outer(A, S1) + np.outer(S1, A)) * c1
                                          + S2 * c2)
        return self.c * out.reshape(n * nu, n * nu)

    def local(self, epsrel=1e-11, epsabs=0.0):
        J = np.array([self.Vk[1] - self.Vk[0], self.Vk[2] - self.Vk[0]]).T
        detJ = abs(np.linalg.det(J))

        def f2(x2, x1):
            x = self.Vk[0] + J @ np.array([x1, x2])
            return self.inner(x)

        def f1(x1):
            r, _ = quad_vec(lambda x2: f2(x2, x1), 0.0, 1.0 - x1, epsrel=epsrel, epsabs=epsabs)
            return r

        res, _ = quad_vec(f1, 0.0, 1.0, epsrel=epsrel, epsabs=epsabs)
        return self.union, detJ * res


class PolarPairIntegral:
    """The same local matrix by a second route that also covers the
    hypersingular kernel c |z|^-3 (s = 1/2, Sec. 3.1): for every outer point
    x the inner integral is taken in polar coordinates y = x + r e(theta).
    Along a ray the basis differences are affine in r,
        a_u(x, y) = A_u(x) - r g_u . e,
    with A_u = phi^k_u(x) - phi^l_u(x) (phi^l extended affinely to x) and g_u
    the gradient of T_l's basis, so the r-integral over the ray's chord
    [r1, r2] of T_l is closed-form:
        int (A_a - r ga)(A_b - r gb) r^(1 - alpha) dr
    (terms r^p with p = -2, -1, 0 for alpha = 3; log for p = -1).  theta is
    integrated by 40-point Gauss-Legendre between the directions of T_l's
    vertices, x by scipy's adaptive quad_vec.  For x inside T_l (identical
    pairs) A = 0 and r1 = 0."""

    def __init__(self, Vk, Vl, nodes_k, nodes_l, kernel, c):
        base = PairIntegral(Vk, Vl, nodes_k, nodes_l, "constant", c)
        self.Vk, self.Vl, self.Gk, self.Gl = base.Vk, base.Vl, base.Gk, base.Gl
        self.Nl, self.Cl = base.Nl, base.Cl
        self.union, self.ink, self.inl = base.union, base.ink, base.inl
        self.identical = sorted(nodes_k) == sorted(nodes_l)
        self.alpha = {"constant": 0, "inv_dist": 1, "peridynamic": 1, "frac_half": 3}[kernel]
        self.ncomp = 2 if kernel == "peridynamic" else 1
        self.c = c

    @staticmethod
    def _ipow(p, r1, r2):
        if p == -1:
            return np.log(r2 / r1)
        return (r2 ** (p + 1) - r1 ** (p + 1)) / (p + 1)

    def _theta_nodes(self, x):
        ang = np.arctan2(self.Vl[:, 1] - x[1], self.Vl[:, 0] - x[0])
        if self.identical:
            cuts = np.sort(np.mod(ang, 2 * np.pi))
            cuts = np.concatenate([cuts, [cuts[0] + 2 * np.pi]])
        else:
            ref = np.arctan2(*(self.Vl.mean(axis=0) - x)[::-1])
            rel = np.mod(ang - ref + np.pi, 2 * np.pi) - np.pi
            cuts = ref + np.sort(rel)
        th, wt = [], []
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            th.append(0.5 * (hi - lo) * _GX + 0.5 * (hi + lo))
            wt.append(0.5 * (hi - lo) * _GW)
        return np.concatenate(th), np.concatenate(wt)

    def inner(self, x):
        pk = _phi(self.Vk, self.Gk, x)
        pl = _phi(self.Vl, self.Gl, x)
        nu = len(self.union)
        A = np.zeros(nu)
        Gr = np.zeros((nu, 2))
        for u in range(nu):
            fx = pk[self.ink[u]] if self.ink[u] >= 0 else 0.0
            py = pl[self.inl[u]] if self.inl[u] >= 0 else 0.0
            A[u] = fx - py
            if self.inl[u] >= 0:
                Gr[u] = self.Gl[self.inl[u]]
        th, wt = self._theta_nodes(x)
        e = np.stack([np.cos(th), np.sin(th)], axis=1)            # (T, 2)
        ne = e @ self.Nl.T                                         # (T, 3)
        gap = self.Cl - self.Nl @ x                                # (3,)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = gap[None, :] / ne
        r2 = np.min(np.where(ne > 0, t, np.inf), axis=1)
        r1 = np.max(np.where(ne < 0, t, 0.0), axis=1)
        r1 = np.maximum(r1, 0.0)
        keep = r2 > r1
        th, wt, e, r1, r2 = th[keep], wt[keep], e[keep], r1[keep], r2[keep]
        ge = e @ Gr.T                                              # (T, nu): g_u . e
        p0 = 1 - self.alpha
        if self.identical:
            assert np.abs(A).max() < 1e-12
            I0 = I1 = np.zeros_like(r1)
        else:
            I0 = self._ipow(p0, r1, r2)
        I1 = self._ipow(p0 + 1, r1, r2) if not self.identical else I1
        I2 = self._ipow(p0 + 2, r1, r2)
        n = self.ncomp
        out = np.zeros((nu, n, nu, n))
        for cc in range(n):
            for dd in range(n):
                kw = wt if n == 1 else wt * e[:, cc] * e[:, dd]
                S0 = np.sum(kw * I0)
                S1 = (kw * I1) @ ge
                S2 = (ge * (kw * I2)[:, None]).T @ ge
                out[:, cc, :, dd] += np.outer(A, A) * S0 - (np.outer(A, S1) + np.outer(S1, A)) + S2
        return self.c * out.reshape(n * nu, n * nu)

    def local(self, epsrel=1e-10, epsabs=0.0):
        J = np.array([self.Vk[1] - self.Vk[0], self.Vk[2] - self.Vk[0]]).T
        detJ = abs(np.linalg.det(J))

        def f1(x1):
            r, _ = quad_vec(lambda x2: self.inner(self.Vk[0] + J @ np.array([x1, x2])), 0.0, 1.0 - x1,
                            epsrel=epsrel, epsabs=epsabs)
            return r

        res, _ = quad_vec(f1, 0.0, 1.0, epsrel=epsrel, epsabs=epsabs)
        return self.union, detJ * res
