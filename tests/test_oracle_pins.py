"""Pins of the CPU oracle against closed forms, textbook identities, an
independent integrator and brute force (no GPU).

Each test names the part of the oracle it pins and what it is pinned to;
none of them re-derives the oracle's own formula.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from inputs import square_mesh, gauss7, paper7, centroid1, collapsed
from inputs.workloads import small_constant

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cfg(kernel="constant", c=1.0, delta=0.1, approach="bary", rule=None,
        singular_n=0, polygon_n=32):
    rule = rule or gauss7()
    return dict(kernel=kernel, c=c, delta=delta, approach=approach, outer=rule,
                inner=rule, singular_n=singular_n, polygon_n=polygon_n,
                ncomp=2 if kernel == "peridynamic" else 1)


def dense(P, rp, col, val):
    M = P.V.shape[0] * P.n
    return sp.csr_matrix((val, col, rp), shape=(M, M)).toarray()


def mass_matrix(mesh):
    """Textbook P1 mass matrix: |T|/12 (1 + delta_ij) per element."""
    M = mesh.n_vertices
    A = np.zeros((M, M))
    m = np.zeros(M)
    for e in mesh.elements:
        v = mesh.vertices[e]
        area = 0.5 * abs((v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) -
                         (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]))
        for a in range(3):
            m[e[a]] += area / 3.0
            for b in range(3):
                A[e[a], e[b]] += area / 12.0 * (2.0 if a == b else 1.0)
    return A, m


# ----------------------------------------------------------------------
# pair lists: brute force == breadth-first traversal (Alg. 2)

@pytest.mark.parametrize("case", ["const_bary", "invdist_duffy", "poly", "peri", "inf"])
def test_pairs_bruteforce_equals_bfs(oracle_lib, case):
    if case == "const_bary":
        w = small_constant()
        mesh, c = w["mesh"], w
    elif case == "invdist_duffy":
        mesh = square_mesh(14, delta=0.2, jitter=0.2, seed=1)
        c = cfg("inv_dist", delta=0.2, singular_n=5)
    elif case == "poly":
        mesh = square_mesh(12, delta=0.15, jitter=0.1, seed=2)
        c = cfg("constant", delta=0.15, approach="poly")
    elif case == "inf":
        mesh = square_mesh(12, delta=0.15, jitter=0.15, seed=4)
        c = cfg("inv_dist", delta=0.15, approach="inf", singular_n=5)
    else:
        mesh = square_mesh(12, delta=0.25, jitter=0.15, seed=3)
        c = cfg("peridynamic", delta=0.25, singular_n=5)
    P = oracle_lib.Problem(mesh, c)
    k, l, cls = P.pairs()
    kb, lb, cb = P.pairs_bfs()
    assert len(k) > 0
    assert np.array_equal(k, kb) and np.array_equal(l, lb) and np.array_equal(cls, cb)
    # sorted by (k, l), labels admissible
    key = k.astype(np.int64) * mesh.n_elements + l
    assert np.all(np.diff(key) > 0)
    lab = mesh.labels
    assert np.all((lab[k] == 1) | (lab[l] == 1))


def test_pair_count_small_constant(oracle_lib):
    """Counts of the 800-triangle constant-kernel case: 12,906 ordered
    pairs, 6,975 nonzeros over 225 degrees of freedom."""
    w = small_constant()
    P = oracle_lib.Problem(w["mesh"], w)
    k, l, c = P.pairs()
    assert len(k) == 12906
    rp, col = P.pattern(k, l)
    assert len(col) == 6975
    assert int(P.isdof().sum()) == 225


def test_table1_dispatch(oracle_lib):
    """Table 1: touching pairs get the regularising transform when the kernel
    is treated as singular; disjoint pairs always the standard rule."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_dispatch.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows[0] == ["s<=-1", "std", "std"]
    assert all(r[2] == "std" for r in rows)
    mesh = square_mesh(8, delta=0.3)
    E = mesh.elements
    for ns, kern in ((0, "constant"), (5, "inv_dist")):
        P = oracle_lib.Problem(mesh, cfg(kern, delta=0.3, singular_n=ns))
        k, l, cls = P.pairs()
        shared = np.array([len(set(E[a]) & set(E[b])) for a, b in zip(k, l)])
        if ns == 0:
            assert np.all(cls == 0)
        else:
            assert np.array_equal(cls, shared)


# ----------------------------------------------------------------------
# hand-computed asymmetric inclusion (barycentre ball, Sec. 2.2)

def test_two_triangles_by_hand(oracle_lib):
    """T0 = (0,0),(1,0),(0,1), T1 = (3,0),(4,0),(3,1), delta = 2.5, c = 1,
    paper's 7-point rule on both sides.  Distances from the rule points of
    T0 to bary(T1) = (10/3, 1/3): only the vertex (1,0) is within 2.5
    (|.|^2 = 50/9 < 6.25); from T1's points to bary(T0) = (1/3, 1/3) the
    nearest is (3, 1/2) with |.|^2 = 257/36 > 6.25.  So (0,1) is a pair,
    (1,0) is not, and with d_p = 1/40 for that vertex
      A1 = d_p * 1/2 e1 e1^T, A2 = -d_p e1 (1/6, 1/6, 1/6),
      A3 = d_p * (1 + delta_ij)/24.
    Self pairs see the whole element: c (2|T| M - 2 m m^T) with
    M = (1 + delta_ij)/24, m = 1/6."""
    from inputs.meshes import Mesh
    V = np.array([[0, 0], [1, 0], [0, 1], [3, 0], [4, 0], [3, 1]], float)
    E = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    mesh = Mesh(V, E, np.array([1, 1], np.int32), 1.0, 1, 0)
    P = oracle_lib.Problem(mesh, cfg("constant", c=1.0, delta=2.5, rule=paper7()))
    k, l, cls = P.pairs()
    assert list(zip(k, l)) == [(0, 0), (0, 1), (1, 1)]
    F = Fraction
    L01 = [[F(0)] * 6 for _ in range(6)]
    dp = F(1, 40)
    L01[1][1] = dp * F(1, 2)
    for j in range(3):
        L01[1][3 + j] = -dp * F(1, 6)
        L01[3 + j][1] = -dp * F(1, 6)
        for i in range(3):
            L01[3 + i][3 + j] = dp * F(2 if i == j else 1, 24)
    nodes, L = P.local(0, 1, 0)
    assert list(nodes) == [0, 1, 2, 3, 4, 5]
    assert np.max(np.abs(L - np.array(L01, dtype=float))) < 1e-16
    self_blk = np.array([[float(F(2 if i == j else 1, 24) - F(1, 18)) for j in range(3)]
                         for i in range(3)])
    A = dense(P, *P.assemble())
    expect = np.array(L01, dtype=float)
    expect[:3, :3] += self_blk
    expect[3:, 3:] += self_blk
    assert np.max(np.abs(A - expect)) < 1e-15


# ----------------------------------------------------------------------
# constant kernel, every pair fully interacting: closed form

@pytest.mark.parametrize("singular_n", [0, 5])
@pytest.mark.parametrize("rule", ["gauss7", "paper7"])
def test_constant_kernel_full_ball_closed_form(oracle_lib, singular_n, rule):
    """With the ball covering the whole mesh, A(phi_j, phi_i) =
    c int int (phi_i(x)-phi_i(y))(phi_j(x)-phi_j(y)) = c (2|D| M_ij - 2 m_i m_j)
    (M the P1 mass matrix, m_i = int phi_i) for every degree of freedom i;
    both the product rule and the touching-pair transforms are exact here."""
    mesh = square_mesh(5, m=1, jitter=0.2, seed=4)
    r = gauss7() if rule == "gauss7" else paper7()
    c = 3.7
    P = oracle_lib.Problem(mesh, cfg("constant", c=c, delta=100.0, rule=r, singular_n=singular_n))
    A = dense(P, *P.assemble())
    M, m = mass_matrix(mesh)
    D = m.sum()
    expect = c * (2 * D * M - 2 * np.outer(m, m))
    dof = P.isdof()
    assert np.max(np.abs(A[dof] - expect[dof])) < 1e-13 * np.abs(expect).max()
    assert np.all(A[~dof] == 0)


def test_constant_kernel_touching_transform_equals_product_rule(oracle_lib):
    """For the constant kernel the integrand is a polynomial of degree 2, so
    the transforms to (0,1)^4 and the 7x7 product rule must agree."""
    mesh = square_mesh(4, m=1, jitter=0.2, seed=5)
    Pd = oracle_lib.Problem(mesh, cfg("constant", delta=100.0, singular_n=5))
    Ps = oracle_lib.Problem(mesh, cfg("constant", delta=100.0, singular_n=0))
    k, l, cls = Pd.pairs()
    seen = set()
    for a, b, c in zip(k, l, cls):
        if c == 0 or c in seen and len(seen) == 3:
            continue
        seen.add(int(c))
        n1, L1 = Pd.local(a, b, c)
        n2, L2 = Ps.local(a, b, 0)
        assert list(n1) == sorted(n1, key=list(n2).index) or set(n1) == set(n2)
        perm = [list(n2).index(x) for x in n1]
        L2p = L2[np.ix_(perm, perm)]
        assert np.max(np.abs(L1 - L2p)) < 1e-14 * np.abs(L2).max()
    assert seen == {1, 2, 3}


# ----------------------------------------------------------------------
# regularising transforms (Sec. 2.4.2): cubature on T x T

def _tri_int(a, b):
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("cls", [1, 2, 3])
def test_touching_transforms_are_cubatures(oracle_lib, cls):
    """Every transform maps (0,1)^4 onto T^ x T^ with the right Jacobian:
    weights sum to |T^|^2 = 1/4, samples lie in T^ x T^ and all monomials of
    total degree <= 3 in (xi, eta) integrate exactly."""
    xi, eta, w = oracle_lib.duffy_samples(cls, 5)
    assert abs(w.sum() - 0.25) < 1e-15
    for p in (xi, eta):
        assert p.min() >= -1e-15 and (p.sum(axis=1)).max() <= 1 + 1e-15
    worst = 0.0
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                for d in range(4 - a - b - c):
                    q = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * eta[:, 0] ** c * eta[:, 1] ** d)
                    ex = _tri_int(a, b) * _tri_int(c, d)
                    worst = max(worst, abs(q - ex))
    assert worst < 2e-16


def _touching_examples(mesh, E, k0):
    pick = {}
    for l in range(len(E)):
        s = len(set(E[k0]) & set(E[l]))
        if s and s not in pick:
            pick[s] = l
        if s == 0 and 0 not in pick:
            v = mesh.vertices
            if np.linalg.norm(v[E[l]].mean(0) - v[E[k0]].mean(0)) > 2.5 * mesh.h:
                pick[0] = l
    return pick


@pytest.mark.slow
@pytest.mark.parametrize("kernel", ["inv_dist", "peridynamic"])
def test_singular_quadrature_vs_independent_integral(oracle_lib, kernel):
    """Touching pairs: the oracle's transforms converge (n = 16) to an
    independent polar/sinh-transformed integral to 1e-10, and the paper's
    n = 5 rule stays within the quadrature error of that integral."""
    from _refint import PairIntegral
    mesh = square_mesh(4, m=1, jitter=0.2, seed=3)
    E, V = mesh.elements, mesh.vertices
    k0 = 14
    pick = _touching_examples(mesh, E, k0)
    n = 2 if kernel == "peridynamic" else 1
    bound5 = {1: 1e-5, 2: 2e-4, 3: 2e-3}
    for cls in (1, 2, 3):
        l = pick[cls]
        un, Lr = PairIntegral(V[E[k0]], V[E[l]], list(E[k0]), list(E[l]), kernel, 1.0).local(epsrel=1e-12)
        for ns, tol in ((16, 1e-10), (5, bound5[cls])):
            P = oracle_lib.Problem(mesh, cfg(kernel, delta=10.0, singular_n=ns))
            nodes, Lo = P.local(k0, l, cls)
            perm = [un.index(a) for a in nodes]
            idx = np.array([n * p + c for p in perm for c in range(n)])
            R = Lr[np.ix_(idx, idx)]
            err = np.linalg.norm(Lo - R) / np.linalg.norm(R)
            assert err < tol, (cls, ns, err)


def test_fractional_kernel_vs_polar_integral(oracle_lib):
    """Kernel c/|z|^3 (s = 1/2, Sec. 3.1) against the polar-coordinate
    integrals of tests/_refint.py (closed form along each ray, the
    hypersingular terms included): a far pair with a degree-11 product rule
    and a vertex-touching pair with the n = 16 transforms, both to 1e-8.  The
    transforms converge in n: n = 16 and n = 24 agree to 1e-8 on all three
    touching classes.  (The identical and edge pairs agree with the polar
    route to 2e-6 and 9e-7, within that route's own theta-quadrature error;
    at about a minute each those runs are not part of the suite.)"""
    from _refint import PolarPairIntegral
    mesh = square_mesh(4, m=1, jitter=0.2, seed=3)
    E, V = mesh.elements, mesh.vertices
    k0 = 14
    pick = _touching_examples(mesh, E, k0)
    for cls, ns, tol in ((0, 0, 1e-8), (1, 16, 1e-8)):
        l = pick[cls]
        un, Lp = PolarPairIntegral(V[E[k0]], V[E[l]], list(E[k0]), list(E[l]), "frac_half", 1.0).local(epsrel=1e-7)
        c = cfg("frac_half", delta=10.0, singular_n=ns, rule=collapsed(6) if cls == 0 else None)
        nodes, Lo = oracle_lib.Problem(mesh, c).local(k0, l, cls)
        perm = [un.index(a) for a in nodes]
        R = Lp[np.ix_(perm, perm)]
        assert np.linalg.norm(Lo - R) / np.linalg.norm(R) < tol, (cls, np.linalg.norm(Lo - R) / np.linalg.norm(R))
    for cls in (1, 2, 3):
        l = pick[cls]
        L16 = oracle_lib.Problem(mesh, cfg("frac_half", delta=10.0, singular_n=16)).local(k0, l, cls)[1]
        L24 = oracle_lib.Problem(mesh, cfg("frac_half", delta=10.0, singular_n=24)).local(k0, l, cls)[1]
        assert np.linalg.norm(L16 - L24) / np.linalg.norm(L24) < 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("kernel", ["inv_dist", "peridynamic"])
def test_far_pair_integrand_vs_independent_integral(oracle_lib, kernel):
    """Disjoint pair, ball covering both: with a degree-11 product rule the
    oracle's truncation quadrature converges to the exact integral."""
    from _refint import PairIntegral
    mesh = square_mesh(4, m=1, jitter=0.2, seed=3)
    E, V = mesh.elements, mesh.vertices
    k0 = 14
    l = _touching_examples(mesh, E, k0)[0]
    n = 2 if kernel == "peridynamic" else 1
    un, Lr = PairIntegral(V[E[k0]], V[E[l]], list(E[k0]), list(E[l]), kernel, 1.0).local(epsrel=1e-12)
    P = oracle_lib.Problem(mesh, cfg(kernel, delta=10.0, rule=collapsed(6)))
    nodes, Lo = P.local(k0, l, 0)
    perm = [un.index(a) for a in nodes]
    idx = np.array([n * p + c for p in perm for c in range(n)])
    R = Lr[np.ix_(idx, idx)]
    assert np.linalg.norm(Lo - R) / np.linalg.norm(R) < 1e-9


# ----------------------------------------------------------------------
# global invariants (Remark on symmetry; null space of the Neumann case)

def _problem(oracle_lib, which):
    if which == "const":
        w = small_constant()
        return oracle_lib.Problem(w["mesh"], w), w["mesh"]
    if which == "invdist":
        mesh = square_mesh(16, delta=0.15, jitter=0.2, seed=0)
        return oracle_lib.Problem(mesh, cfg("inv_dist", c=2.0, delta=0.15, singular_n=5)), mesh
    if which == "poly":
        mesh = square_mesh(12, delta=0.15, jitter=0.15, seed=0)
        return oracle_lib.Problem(mesh, cfg("constant", c=2.0, delta=0.15, approach="poly")), mesh
    if which == "frac":
        mesh = square_mesh(12, delta=0.2, jitter=0.2, seed=0)
        return oracle_lib.Problem(mesh, cfg("frac_half", c=2.0, delta=0.2, singular_n=5)), mesh
    if which == "inf":
        mesh = square_mesh(12, delta=0.15, jitter=0.2, seed=0)
        return oracle_lib.Problem(mesh, cfg("inv_dist", c=2.0, delta=0.15, approach="inf", singular_n=5)), mesh
    mesh = square_mesh(12, delta=0.2, jitter=0.15, seed=0)
    return oracle_lib.Problem(mesh, cfg("peridynamic", c=2.0, delta=0.2, singular_n=5)), mesh


@pytest.mark.parametrize("which", ["const", "invdist", "poly", "peri", "frac", "inf"])
def test_symmetry_and_null_space(oracle_lib, which):
    P, mesh = _problem(oracle_lib, which)
    rp, col, val = P.assemble()
    A = sp.csr_matrix((val, col, rp), shape=(P.n * mesh.n_vertices,) * 2)
    dofm = np.repeat(P.isdof(), P.n)
    B = A[dofm][:, dofm]
    asym = abs(B - B.T).max() / abs(B).max()
    assert asym < 1e-14
    absrow = np.asarray(abs(A).sum(axis=1)).ravel()
    X, Y = mesh.vertices[:, 0], mesh.vertices[:, 1]
    if P.n == 1:
        modes = [np.ones(mesh.n_vertices)]
    else:
        ones, zeros = np.ones_like(X), np.zeros_like(X)
        modes = [np.stack([ones, zeros], 1).ravel(), np.stack([zeros, ones], 1).ravel(),
                 np.stack([-Y, X], 1).ravel()]
    for U in modes:
        r = A @ U
        scale = np.asarray(abs(A) @ abs(U)).ravel()
        ok = dofm
        assert np.all(np.abs(r[ok]) <= 1e-13 * scale[ok] + 1e-300)


def test_translation_invariance_uniform_mesh(oracle_lib):
    """On the uniform mesh every interior degree of freedom sees a translated
    copy of the same neighbourhood, and the mesh and the symmetric 7-point
    rule are invariant under point reflection through a node: A u = 0 for
    linear u, and A u is the same in every interior row for quadratic u."""
    P, mesh = _problem(oracle_lib, "const")
    rp, col, val = P.assemble()
    A = sp.csr_matrix((val, col, rp), shape=(mesh.n_vertices,) * 2)
    X, Y = mesh.vertices[:, 0], mesh.vertices[:, 1]
    h = mesh.h
    interior = P.isdof() & (X > 3 * h - 1e-12) & (X < 1 - 3 * h + 1e-12) & \
        (Y > 3 * h - 1e-12) & (Y < 1 - 3 * h + 1e-12)
    assert interior.sum() >= 25
    scale = abs(A).max()
    for U in (X, Y, 2 * X - 3 * Y):
        assert np.abs((A @ U)[interior]).max() < 1e-12 * scale
    q = (A @ (X ** 2 + Y ** 2))[interior]
    assert np.ptp(q) < 1e-12 * scale
    q2 = (A @ (X * Y))[interior]
    assert np.ptp(q2) < 1e-12 * scale


# ----------------------------------------------------------------------
# 32-gon ball (Def. 2.4 reading): clipping and sub-triangle quadrature

def test_polygon_inner_moments(oracle_lib):
    """Summed over all inner elements, the clipped-and-retriangulated inner
    quadrature reproduces the moments of the regular N-gon P around x:
    |P| = N/2 delta^2 sin(2pi/N), int y = |P| x, and
    int (y-x)(y-x)^T = N delta^4 sin(2pi/N)(2 + cos(2pi/N))/24 * I.
    The trace ratio to the disc is kappa_32 = 0.98722302."""
    N, delta = 32, 0.12
    mesh = square_mesh(10, delta=delta, jitter=0.2, seed=6)
    P = oracle_lib.Problem(mesh, cfg("constant", delta=delta, approach="poly", polygon_n=N))
    th = 2 * math.pi / N
    area = 0.5 * N * delta ** 2 * math.sin(th)
    I2 = N * delta ** 4 * math.sin(th) * (2 + math.cos(th)) / 24.0
    kappa = I2 / (math.pi * delta ** 4 / 4)
    assert abs(kappa - 0.98722302) < 1e-8
    rng = np.random.default_rng(7)
    V, E = mesh.vertices, mesh.elements
    for x in rng.uniform(0.05, 0.95, size=(12, 2)):
        tot0, tot1, tot2 = 0.0, np.zeros(2), np.zeros((2, 2))
        nclipped = 0
        for l in range(mesh.n_elements):
            a0, a1, a2 = P.inner_moments(x, l)
            if a0 == 0.0:
                continue
            v = V[E[l]]
            tot0 += a0
            tot1 += a1 @ v
            tot2 += v.T @ a2 @ v
            if abs(a0 - 0.5 * abs(np.linalg.det(np.array([v[1] - v[0], v[2] - v[0]])))) > 1e-15:
                nclipped += 1
        assert nclipped > 5
        assert abs(tot0 - area) < 1e-14
        assert np.abs(tot1 - area * x).max() < 1e-14
        cen = tot2 - area * np.outer(x, x)
        assert np.abs(cen - I2 * np.eye(2)).max() < 1e-15


def test_polygon_clip_area_matches_shoelace_sum(oracle_lib):
    """Clip areas of all inner elements add up to the polygon area."""
    N, delta = 32, 0.1
    mesh = square_mesh(8, delta=delta, seed=0)
    P = oracle_lib.Problem(mesh, cfg("constant", delta=delta, approach="poly", polygon_n=N))
    x = np.array([0.43, 0.57])
    s = sum(P.clip_area(x, l)[0] for l in range(mesh.n_elements))
    assert abs(s - 0.5 * N * delta ** 2 * math.sin(2 * math.pi / N)) < 1e-15


# ----------------------------------------------------------------------
# load vector

def test_rhs_closed_forms(oracle_lib):
    """Both rules integrate linear forcing times P1 exactly:
    b_i = sum_{T in Omega, T ni i} sum_j f(v_j) |T|/12 (1 + delta_ij)."""
    mesh = square_mesh(8, delta=0.2, jitter=0.2, seed=8)
    for r in (gauss7(), paper7()):
        P = oracle_lib.Problem(mesh, cfg("constant", delta=0.2, rule=r))
        b = P.rhs(f_const=[-4.0])
        Mfull, _ = mass_matrix(mesh)
        from inputs.meshes import Mesh
        om = Mesh(mesh.vertices, mesh.elements[mesh.labels == 1], mesh.labels[mesh.labels == 1],
                  mesh.h, mesh.n, mesh.m)
        Mo, mo = mass_matrix(om)
        assert np.abs(b - (-4.0) * mo).max() < 1e-15
        f = 0.5 - 2.0 * mesh.vertices[:, 0] + 3.0 * mesh.vertices[:, 1]
        b2 = P.rhs(f_affine=[(0.5, -2.0, 3.0)])
        assert np.abs(b2 - Mo @ f).max() < 1e-15
    # vector case: components independent
    P = oracle_lib.Problem(mesh, cfg("peridynamic", delta=0.2, singular_n=5))
    b = P.rhs(f_affine=[(-1.0, -2.0, 0.0), (0.0, 0.0, -1.0)])
    f0 = -1.0 - 2.0 * mesh.vertices[:, 0]
    f1 = -mesh.vertices[:, 1]
    assert np.abs(b[0::2] - Mo @ f0).max() < 1e-15
    assert np.abs(b[1::2] - Mo @ f1).max() < 1e-15


def test_masked_pair_search_is_a_filter(oracle_lib):
    """The row-restricted search (used for sampled rows of large meshes)
    lists exactly the pairs of the full search that meet a masked element."""
    from inputs.workloads import inv_dist_jittered
    w = inv_dist_jittered(n=16, delta=0.15, precision="fp64")
    mesh = w["mesh"]
    P = oracle_lib.Problem(mesh, w)
    k, l, c = P.pairs()
    rng = np.random.default_rng(3)
    mask = np.zeros(mesh.n_elements, bool)
    mask[rng.choice(mesh.n_elements, 25, replace=False)] = True
    mk, ml, mc = P.pairs(elem_mask=mask)
    keep = mask[k] | mask[l]
    assert np.array_equal(mk, k[keep]) and np.array_equal(ml, l[keep]) and np.array_equal(mc, c[keep])


def _exact_quadratic_load(mesh, quad):
    """b_i = sum over Omega elements T containing i of the exact integral of
    q(x) phi_i(x) over T, for q(x) = sum_ab quad[a][b] x_a x_b: with
    x = sum_j lambda_j v_j the integrand is a cubic in the barycentric
    coordinates, integrated by the closed form
    int_T l1^a l2^b l3^c = 2|T| a! b! c! / (a+b+c+2)!."""
    from math import factorial
    b = np.zeros(mesh.n_vertices)
    for e in np.nonzero(mesh.labels == 1)[0]:
        v = mesh.vertices[mesh.elements[e]]
        area = 0.5 * abs(np.cross(v[1] - v[0], v[2] - v[0]))
        for i in range(3):
            s = 0.0
            for j in range(3):
                for k in range(3):
                    ex = [0, 0, 0]
                    ex[i] += 1
                    ex[j] += 1
                    ex[k] += 1
                    mono = 2 * area * np.prod([factorial(t) for t in ex]) / factorial(5)
                    s += mono * sum(quad[a][c] * v[j][a] * v[k][c] for a in range(2) for c in range(2))
            b[mesh.elements[e][i]] += s
    return b


def test_rhs_quadrature_point_values_closed_form(oracle_lib):
    """The load vector from values at the outer quadrature points: with the
    degree-5 rule, quadratic forcing times P1 is integrated exactly, so b
    equals the closed form above for f sampled at the points the rule maps to
    each element (one function per component for the vector case)."""
    mesh = square_mesh(6, delta=0.2, jitter=0.2, seed=4)
    r = gauss7()
    V, E = mesh.vertices, mesh.elements
    v0 = V[E[:, 0]]
    J = np.stack([V[E[:, 1]] - v0, V[E[:, 2]] - v0], axis=2)
    X = v0[:, None, :] + np.einsum("kij,pj->kpi", J, r.xi)           # [K, P, 2]
    qa = [[1.0, -1.5], [-1.5, 0.0]]    # x^2 - 3 x y
    qb = [[0.0, 0.5], [0.5, 2.0]]      # x y + 2 y^2
    fa = X[..., 0] ** 2 - 3.0 * X[..., 0] * X[..., 1]
    fb = X[..., 0] * X[..., 1] + 2.0 * X[..., 1] ** 2
    P = oracle_lib.Problem(mesh, cfg("constant", delta=0.2, rule=r))
    b = P.rhs(f_qp=fa[..., None])
    ea = _exact_quadratic_load(mesh, qa)
    assert np.abs(b - ea).max() <= 1e-15 * max(1.0, np.abs(ea).max())
    Pv = oracle_lib.Problem(mesh, cfg("peridynamic", delta=0.2, singular_n=5, rule=r))
    bv = Pv.rhs(f_qp=np.stack([fa, fb], axis=-1))
    assert np.abs(bv[0::2] - ea).max() <= 1e-15 * max(1.0, np.abs(ea).max())
    eb = _exact_quadratic_load(mesh, qb)
    assert np.abs(bv[1::2] - eb).max() <= 1e-15 * max(1.0, np.abs(eb).max())
    # paper7 is exact to degree 3 only: the same check holds for it too
    # (quadratic f times P1 is cubic)
    r7 = paper7()
    X7 = v0[:, None, :] + np.einsum("kij,pj->kpi", J, r7.xi)
    f7 = X7[..., 0] ** 2 - 3.0 * X7[..., 0] * X7[..., 1]
    P7 = oracle_lib.Problem(mesh, cfg("constant", delta=0.2, rule=r7))
    assert np.abs(P7.rhs(f_qp=f7[..., None]) - ea).max() <= 1e-15 * max(1.0, np.abs(ea).max())


def _scale_problem(oracle_lib, n, approach, delta=0.25):
    from inputs.workloads import c_frac
    mesh = square_mesh(n, delta=delta)
    P = oracle_lib.Problem(mesh, cfg("constant", c=c_frac(-1.0, delta), delta=delta, approach=approach))
    rp, col, val = P.assemble()
    M = mesh.n_vertices
    A = sp.csr_matrix((val, col, rp), shape=(M, M))
    u = mesh.vertices[:, 0] ** 2 + mesh.vertices[:, 1] ** 2
    return mesh, P, A, u, P.isdof()


def _manufactured_solve(P, A, u, dof, f):
    """Solve A_dd U_d = b_d - A_db u_b (nonlocal Dirichlet data u on the
    layer, Sec. 3 eq. inhomogeneousDirichletData) and return max |U - u| at
    the degrees of freedom."""
    import scipy.sparse.linalg as spla
    Add = A[dof][:, dof].tocsc()
    Adb = A[dof][:, ~dof]
    b = P.rhs(f_const=[f])
    x = spla.spsolve(Add, b[dof] - Adb @ u[~dof])
    return float(np.abs(x - u[dof]).max())


@pytest.mark.parametrize("n", [8, 16])
def test_operator_scale_polygon_uniform_mesh(oracle_lib, n):
    """The absolute scale of the whole assembly (factor 2 of the weak form,
    kernel constant 4/(pi delta^4), four terms, Sec. 2.1 and 3.1).  With the
    inscribed N-gon and a rule exact on quadratics, the continuous identity
    2c int_P (u(x) - u(y)) dy = -kappa_N Delta u holds exactly for quadratic
    u; on a uniform mesh the interpolation error of u is lattice-periodic and
    the form annihilates it against a hat function (translation invariance
    and constants in the null space), so at EVERY degree of freedom
    (A I_h u)_i = -4 kappa_N int phi_i exactly for u = |x|^2, with
    kappa_32 = 32 sin(2 pi/32)(2 + cos(2 pi/32))/(6 pi).  Consequently the
    manufactured solve with f = -4 kappa_N reproduces u at the nodes."""
    kappa = 32 * math.sin(2 * math.pi / 32) * (2 + math.cos(2 * math.pi / 32)) / (6 * math.pi)
    assert abs(kappa - 0.98722302) < 1e-8
    mesh, P, A, u, dof = _scale_problem(oracle_lib, n, "poly")
    phi_int = P.rhs(f_const=[1.0])
    ratio = (A @ u)[dof] / (-4.0 * phi_int[dof])
    assert np.abs(ratio - kappa).max() <= 1e-11
    assert _manufactured_solve(P, A, u, dof, -4.0 * kappa) <= 1e-11


def test_manufactured_solution_trend_barycentre(oracle_lib):
    """Manufactured solution u = |x|^2, f = -4 with the barycentre ball on
    uniform meshes at fixed delta (Table 2 style, Sec. 3.1): the nodal error
    of the solve and the deviation of A I_h u from -Delta u tested against the
    hat functions both shrink at least ~h^2 (factor >= 3.5 per halving)."""
    errs, devs = [], []
    for n in (8, 16, 32):
        mesh, P, A, u, dof = _scale_problem(oracle_lib, n, "bary")
        phi_int = P.rhs(f_const=[1.0])
        devs.append(float(np.abs((A @ u)[dof] / (-4.0 * phi_int[dof]) - 1.0).max()))
        errs.append(_manufactured_solve(P, A, u, dof, -4.0))
    assert errs[-1] < 2e-3 and devs[-1] < 1.5e-2
    for a, b in zip(errs, errs[1:]):
        assert a / b >= 3.5, errs
    for a, b in zip(devs, devs[1:]):
        assert a / b >= 3.5, devs


# ----------------------------------------------------------------------
# infinity-norm ball (Def. 2.5): exact square clipping

@pytest.mark.parametrize("n", [8, 16])
def test_operator_scale_inf_ball_uniform_mesh(oracle_lib, n):
    """The square {|x - y|_inf <= delta} is clipped exactly and the rules are
    exact on quadratics, so with c = 3/(4 delta^4) (Sec. 3.3) the continuous
    identity 2c int_square (u(x) - u(y)) dy = -Delta u (the second moment of
    the square is 8 delta^4/3 per axis) holds exactly for quadratic u; on a
    uniform mesh this gives (A I_h u)_i = -4 int phi_i at every degree of
    freedom (as for the N-gon, with kappa = 1), and the manufactured solve
    with f = -4 reproduces u at the nodes."""
    delta = 0.25
    mesh = square_mesh(n, delta=delta)
    P = oracle_lib.Problem(mesh, cfg("constant", c=3.0 / (4.0 * delta ** 4), delta=delta, approach="inf"))
    rp, col, val = P.assemble()
    M = mesh.n_vertices
    A = sp.csr_matrix((val, col, rp), shape=(M, M))
    u = mesh.vertices[:, 0] ** 2 + mesh.vertices[:, 1] ** 2
    dof = P.isdof()
    phi_int = P.rhs(f_const=[1.0])
    ratio = (A @ u)[dof] / (-4.0 * phi_int[dof])
    assert np.abs(ratio - 1.0).max() <= 1e-11
    assert _manufactured_solve(P, A, u, dof, -4.0) <= 1e-11


def _box_triangle_area(v, lo, hi):
    """Area of triangle v inside the box [lo, hi] by integrating the length of
    each vertical slice (an interval of the triangle cut to the box) with
    adaptive quadrature between the breakpoints: independent of polygon
    clipping."""
    from scipy.integrate import quad
    xs = sorted(set([lo[0], hi[0]] + [p[0] for p in v]))

    def slice_len(x):
        ys = []
        for a in range(3):
            p, q = v[a], v[(a + 1) % 3]
            if (p[0] - x) * (q[0] - x) <= 0 and p[0] != q[0]:
                ys.append(p[1] + (x - p[0]) / (q[0] - p[0]) * (q[1] - p[1]))
        if len(ys) < 2:
            return 0.0
        y0, y1 = max(min(ys), lo[1]), min(max(ys), hi[1])
        return max(0.0, y1 - y0)

    a, b = max(lo[0], min(p[0] for p in v)), min(hi[0], max(p[0] for p in v))
    if b <= a:
        return 0.0
    pts = [x for x in xs if a < x < b]
    return quad(slice_len, a, b, points=pts or None, epsabs=1e-15, epsrel=1e-12, limit=200)[0]


def test_inf_ball_clip_area_independent(oracle_lib):
    """Clip areas of T_l and the square around x against slice integration,
    for straddling and inside cases; and summed over a mesh they give the
    square's area 4 delta^2."""
    delta = 0.1
    mesh = square_mesh(8, delta=delta, jitter=0.2, seed=21)
    P = oracle_lib.Problem(mesh, cfg("constant", delta=delta, approach="inf"))
    rng = np.random.default_rng(22)
    V, E = mesh.vertices, mesh.elements
    checked = 0
    for x in rng.uniform(0.1, 0.9, size=(6, 2)):
        tot = 0.0
        for l in range(mesh.n_elements):
            a, _ = P.clip_area(x, l)
            tot += abs(a)
            if a != 0.0 and checked < 60:
                ref = _box_triangle_area(V[E[l]], x - delta, x + delta)
                assert abs(abs(a) - ref) <= 1e-12 * delta ** 2
                checked += 1
        assert abs(tot - 4 * delta ** 2) < 1e-15
    assert checked == 60


def test_inf_ball_convergence_rates_table7(oracle_lib):
    """Table 7 (golden fixture): manufactured solution on Omega = (0, 0.5)^2
    with delta = sqrt(2) h (two cells), 7-point rule of the numerical
    section; the L2 error decreases at the printed rates 2.32 and 2.18 (within
    0.05).  The absolute errors here are a constant factor of about 1.65 above
    the printed ones at every level (the paper does not define the error
    norm it reports), so only the rates are pinned."""
    import scipy.sparse.linalg as spla
    rows = [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, "table7_inf_ball_rates.txt"))
            if l.strip() and not l.startswith("#")]
    errs = []
    for n in (5, 10, 20):
        side = 0.5
        delta = 2 * side / n
        mesh = square_mesh(n, m=2, side=side)
        r = paper7()
        P = oracle_lib.Problem(mesh, cfg("constant", c=3.0 / (4.0 * delta ** 4), delta=delta, approach="inf",
                                         rule=r))
        assert abs(math.sqrt(2) * side / n - rows[len(errs)][0]) < 0.005 * rows[len(errs)][0]
        rp, col, val = P.assemble()
        M = mesh.n_vertices
        A = sp.csr_matrix((val, col, rp), shape=(M, M))
        V, E = mesh.vertices, mesh.elements

        def u(X):
            return np.sin(4 * np.pi * X[..., 0]) * np.sin(4 * np.pi * X[..., 1])

        v0 = V[E[:, 0]]
        J = np.stack([V[E[:, 1]] - v0, V[E[:, 2]] - v0], axis=2)
        X = v0[:, None, :] + np.einsum("kij,pj->kpi", J, r.xi)
        b = P.rhs(f_qp=(32 * np.pi ** 2 * u(X))[..., None])
        dof = P.isdof()
        U = u(V)
        Uh = U.copy()
        Uh[dof] = spla.spsolve(A[dof][:, dof].tocsc(), b[dof] - A[dof][:, ~dof] @ U[~dof])
        g = gauss7()
        Xg = v0[:, None, :] + np.einsum("kij,pj->kpi", J, g.xi)
        lam = np.stack([1 - g.xi[:, 0] - g.xi[:, 1], g.xi[:, 0], g.xi[:, 1]], 1)
        eh = np.einsum("kv,pv->kp", Uh[E], lam) - u(Xg)
        det = np.abs(J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0])
        om = mesh.labels == 1
        errs.append(math.sqrt((det[om, None] * g.w[None, :] * eh[om] ** 2).sum()))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    for got, row in zip(rates, rows[1:]):
        assert abs(got - row[3]) <= 0.05, (rates, [r[3] for r in rows[1:3]])
    for e, row in zip(errs, rows):
        assert 1.5 <= e / row[2] <= 1.8


# ----------------------------------------------------------------------
# the paper's ball approximations (Def. 2.3 nocaps, Def. 2.4 approxcaps)

def _global_hull_area(mesh, x, delta, caps):
    """Area of the convex hull of the crossings of the circle |y - x| = delta
    with ALL mesh edges (Def. 2.3), plus the arc midpoints between
    consecutive crossings (Def. 2.4): the points lie on the circle, so the
    area is delta^2/2 sum sin(angle gaps).  Written from the definitions,
    over the whole mesh, with no per-element construction."""
    V, E = mesh.vertices, mesh.elements
    edges = {tuple(sorted((int(e[i]), int(e[(i + 1) % 3])))) for e in E for i in range(3)}
    ang = []
    for a, b in edges:
        p, d = V[a], V[b] - V[a]
        f = p - x
        A, B, C = d @ d, f @ d, f @ f - delta ** 2
        D = B * B - A * C
        if D <= 0:
            continue
        for t in ((-B - math.sqrt(D)) / A, (-B + math.sqrt(D)) / A):
            if 0.0 <= t <= 1.0:
                y = f + t * d
                ang.append(math.atan2(y[1], y[0]) % (2 * math.pi))
    ang = np.unique(np.round(np.sort(ang), 13))
    if caps:
        nxt = np.concatenate([ang[1:], [ang[0] + 2 * math.pi]])
        ang = np.sort(np.concatenate([ang, 0.5 * (ang + nxt)]))
    gaps = np.diff(np.concatenate([ang, [ang[0] + 2 * math.pi]]))
    return 0.5 * delta ** 2 * np.sin(gaps).sum()


@pytest.mark.parametrize("approach", ["nocaps", "approxcaps"])
def test_caps_balls_are_the_global_hull(oracle_lib, approach):
    """The per-element polygons T_l n B(x) of the oracle add up to the area of
    the hull of Def. 2.3 (resp. 2.4) over the whole mesh, and their area gap
    to the disc is O(h^2) (Sec. 2.2): factor >= 3 per halving of h."""
    delta = 0.13
    rng = np.random.default_rng(5)
    gaps = []
    for n in (10, 20, 40):
        mesh = square_mesh(n, delta=delta, jitter=0.2, seed=31)
        P = oracle_lib.Problem(mesh, cfg("constant", delta=delta, approach=approach))
        worst = 0.0
        for x in rng.uniform(0.2, 0.8, size=(3, 2)):
            near = np.flatnonzero(np.linalg.norm(mesh.vertices[mesh.elements].mean(axis=1) - x, axis=1)
                                  < delta + 2 * mesh.h)
            tot = sum(abs(P.clip_area(x, l)[0]) for l in near)
            assert abs(tot - _global_hull_area(mesh, x, delta, approach == "approxcaps")) < 1e-15
            worst = max(worst, math.pi * delta ** 2 - tot)
        gaps.append(worst)
    assert gaps[0] / gaps[1] >= 3.0 and gaps[1] / gaps[2] >= 3.0, gaps


def _manufactured_l2(oracle_lib, mesh, c_cfg, u, f_affine=None, f_point=None):
    """Solve the nonlocal Dirichlet problem (Sec. 3, eq.
    inhomogeneousDirichletData) with g = u on Omega_D and return
    ||u_h - u||_L2(Omega) by the degree-5 rule and the number of unknowns
    solved for.  u maps points [..., 2] to values [...] (one component) or
    [..., n]; discontinuous unknowns take u at their element's vertex."""
    import scipy.sparse.linalg as spla
    P = oracle_lib.Problem(mesh, c_cfg)
    n = P.n
    rp, col, val = P.assemble()
    N = n * P.n_unknowns
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    V, E = mesh.vertices, mesh.elements
    v0 = V[E[:, 0]]
    J = np.stack([V[E[:, 1]] - v0, V[E[:, 2]] - v0], axis=2)
    if f_point is not None:
        X = v0[:, None, :] + np.einsum("kij,pj->kpi", J, c_cfg["outer"].xi)
        b = P.rhs(f_qp=f_point(X)[..., None])
    else:
        b = P.rhs(f_affine=f_affine)
    uu = lambda X: np.reshape(u(X), X.shape[:-1] + (n,))
    dof = np.repeat(P.isdof(), n)
    U = uu(V[E].reshape(-1, 2) if P.dg else V).reshape(-1)
    Uh = U.copy()
    rhs = b[dof] - A[dof][:, ~dof] @ U[~dof]
    if P.dg:
        Uh[dof] = np.linalg.solve(A[dof][:, dof].toarray(), rhs)
    else:
        Uh[dof] = spla.spsolve(A[dof][:, dof].tocsc(), rhs)
    g = gauss7()
    Xg = v0[:, None, :] + np.einsum("kij,pj->kpi", J, g.xi)
    lam = np.stack([1 - g.xi[:, 0] - g.xi[:, 1], g.xi[:, 0], g.xi[:, 1]], 1)
    Ue = Uh.reshape(-1, 3, n) if P.dg else Uh.reshape(-1, n)[E]
    eh = np.einsum("kvc,pv->kpc", Ue, lam) - uu(Xg)
    det = np.abs(J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0])
    om = mesh.labels == 1
    return math.sqrt((det[om, None, None] * g.w[None, :, None] * eh[om] ** 2).sum()), int(dof.sum())


def _golden_rows(name):
    return [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, name))
            if l.strip() and not l.startswith("#")]


def _u_cubic(X):
    return X[..., 0] ** 2 * X[..., 1] + X[..., 1] ** 2


def _u_navier(X):
    return np.stack([X[..., 1] ** 2, X[..., 0] ** 2 * X[..., 1]], -1)


# f = -(pi/2)(1 + 2 x1, x2) as affine components (a0 + a1 x1 + a2 x2)
_F_NAVIER = [(-math.pi / 2, -math.pi, 0.0), (0.0, 0.0, -math.pi / 2)]


def test_fractional_approxcaps_convergence_table2(oracle_lib):
    """Table 2 (golden fixture): s = 1/2, delta = 0.2, approximate caps, the
    cubic manufactured solution (reproduced by the exact operator, Sec. 3.1)
    on Omega = (0, 0.5)^2 with h = 0.5/5, 0.5/10, 0.5/20 (element diameters
    1.41e-1, 7.07e-2, 3.54e-2; 16, 81, 361 dofs as printed): the L2 error
    decreases at the printed rates 2.13 and 2.01 (within 0.05).  The errors
    here are about 2.0 times the printed ones at every level (the reported
    norm and the meshes are not specified further), so the rates are what is
    pinned; nocaps and the 32-gon give other errors with the same rates."""
    rows = [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, "table2_fractional_rates.txt"))
            if l.strip() and not l.startswith("#")]
    delta = 0.2

    def u(X):
        return X[..., 0] ** 2 * X[..., 1] + X[..., 1] ** 2

    errs = []
    for i, n in enumerate((5, 10, 20)):
        mesh = square_mesh(n, delta=delta, side=0.5)
        c = cfg("frac_half", c=1.0 / (math.pi * delta), delta=delta, approach="approxcaps", rule=paper7(),
                singular_n=5)
        e, ndof = _manufactured_l2(oracle_lib, mesh, c, u, f_affine=[(-2.0, 0.0, -2.0)])
        assert float(f"{ndof:.2e}") == rows[i][1]   # dofs as printed (3 digits)
        errs.append(e)
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    for got, row in zip(rates, rows[1:]):
        assert abs(got - row[3]) <= 0.05, rates
    for e, row in zip(errs, rows):
        assert 1.9 <= e / row[2] <= 2.2, errs


# ----------------------------------------------------------------------
# discontinuous P1 ansatz (three unknowns per element)

@pytest.mark.parametrize("kernel,singular_n", [("constant", 0), ("inv_dist", 5), ("peridynamic", 5),
                                                ("constant", 4), ("frac_half", 5)])
def test_dg_matrix_restricts_to_the_cg_matrix(oracle_lib, kernel, singular_n):
    """A continuous P1 function is a DG function with equal values at shared
    vertices: with P the injection (node, component) -> (3k + a, component)
    over all elements k holding the node, P^T A_DG P = A_CG on the CG degrees
    of freedom (every DG sample and weight is the CG one; the transforms of
    touching pairs included).  The DG matrix is symmetric with zero row
    sums (constants: the sum of all DG basis functions is 1)."""
    mesh = square_mesh(8, delta=0.3, jitter=0.2, seed=3)
    c_cg = cfg(kernel, c=1.5, delta=0.3, singular_n=singular_n)
    Pc = oracle_lib.Problem(mesh, c_cg)
    Pd = oracle_lib.Problem(mesh, dict(c_cg, ansatz="dg"))
    n = Pc.n
    rc, cc, vc = Pc.assemble()
    rd, cd, vd = Pd.assemble()
    Nc, Nd = n * Pc.n_unknowns, n * Pd.n_unknowns
    Ac = sp.csr_matrix((vc, cc, rc), shape=(Nc, Nc))
    Ad = sp.csr_matrix((vd, cd, rd), shape=(Nd, Nd))
    E = mesh.elements
    r = [n * (3 * k + a) + c for k in range(E.shape[0]) for a in range(3) for c in range(n)]
    q = [n * E[k, a] + c for k in range(E.shape[0]) for a in range(3) for c in range(n)]
    P = sp.csr_matrix((np.ones(len(r)), (r, q)), shape=(Nd, Nc))
    dof = np.repeat(Pc.isdof(), n)
    assert abs((P.T @ Ad @ P - Ac).tocsr()[dof]).max() <= 1e-14 * abs(Ac[dof]).max()
    dd = np.repeat(Pd.isdof(), n)
    B = Ad[dd][:, dd]
    assert abs(B - B.T).max() <= 1e-14 * abs(B).max()
    if n == 1:
        assert np.abs(Ad @ np.ones(Nd))[dd].max() <= 1e-13 * abs(Ad).max()
    # rows of Omega_D elements are empty; the load vector has one entry per
    # DG unknown: sum over an element's three entries = int_T f
    assert np.all(np.diff(rd)[np.repeat(~Pd.isdof(), n)] == 0)
    b = Pd.rhs(f_const=[-4.0] * n)
    area = 0.5 * np.abs(np.cross(mesh.vertices[E[:, 1]] - mesh.vertices[E[:, 0]],
                                 mesh.vertices[E[:, 2]] - mesh.vertices[E[:, 0]]))
    bs = b.reshape(-1, 3, n).sum(axis=1)[:, 0]
    assert np.abs(bs - np.where(mesh.labels == 1, -4.0 * area, 0.0)).max() < 1e-15


def test_fractional_dg_convergence_table3(oracle_lib):
    """Table 3 (golden fixture): Table 2's study in the discontinuous space
    (s = 1/2 with jumps across edges: the edge-touching integrals are the
    5-point rule's values).  The mesh labels the two Omega triangles with
    all vertices on the boundary as Omega_D, which gives the printed 144 and
    594 unknowns exactly.  Rates 2.11 and 1.98 against the printed 2.24 and
    1.98 (the first level has 2h > delta, which the paper notes affects the
    first rates); errors about 1.8-2.0 times the printed ones, as for
    Table 2."""
    from inputs import boundary_triangles_to_layer
    rows = _golden_rows("table3_fractional_dg_rates.txt")
    delta = 0.2
    errs = []
    for i, n in enumerate((5, 10, 20)):
        mesh = boundary_triangles_to_layer(square_mesh(n, delta=delta, side=0.5), side=0.5)
        c = dict(cfg("frac_half", c=1.0 / (math.pi * delta), delta=delta, approach="approxcaps", rule=paper7(),
                     singular_n=5), ansatz="dg")
        e, ndof = _manufactured_l2(oracle_lib, mesh, c, _u_cubic, f_affine=[(-2.0, 0.0, -2.0)])
        assert float(f"{ndof:.2e}") == rows[i][1]
        errs.append(e)
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert abs(rates[0] - rows[1][3]) <= 0.15, rates
    assert abs(rates[1] - rows[2][3]) <= 0.05, rates
    for e, row in zip(errs, rows):
        assert 1.7 <= e / row[2] <= 2.2, errs


def test_peridynamic_no_zero_division_convergence_table4(oracle_lib):
    """Table 4 (golden fixture): the peridynamic kernel c zz^T/|z|^3 with the
    paper's c = 3/delta^3 and f = -(pi/2)(1 + 2 x1, x2) (the Navier limit
    operator; the weak form's factor 2 included), delta = 0.1, approximate
    caps, 7-point rule, and touching pairs by the standard rule that avoids
    x_p = y_q (Table 1, s = -1/2; singular_n = 0).  Rates 2.05 and 1.96
    against the printed 2.04 and 1.99, errors 1.23-1.26 times the printed
    ones at every level.  With the regularising transforms instead (which
    overestimate the support on touching pairs when delta ~ h) the coarse
    errors are 15 times larger, so this pins the Table 1 rule, the kernel
    constant and both components of the load vector."""
    rows = _golden_rows("table4_peridynamic_cg_rates.txt")
    delta = 0.1
    errs = []
    for i, n in enumerate((5, 10, 20)):
        mesh = square_mesh(n, delta=delta, side=0.5)
        c = cfg("peridynamic", c=3.0 / delta ** 3, delta=delta, approach="approxcaps", rule=paper7(),
                singular_n=0)
        e, ndof = _manufactured_l2(oracle_lib, mesh, c, _u_navier, f_affine=_F_NAVIER)
        assert float(f"{ndof:.2e}") == rows[i][1]
        errs.append(e)
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    for got, row in zip(rates, rows[1:]):
        assert abs(got - row[3]) <= 0.05, rates
    for e, row in zip(errs, rows):
        assert 1.15 <= e / row[2] <= 1.35, errs


def test_peridynamic_dg_convergence_table5(oracle_lib):
    """Table 5 (golden fixture): Table 4's study in the discontinuous space.
    Unknowns 288 and 1188 as printed (2.88e2, 1.19e3).  The errors converge
    at second order (2.06, 2.05) but the printed rates are lower at these
    levels (1.84, 1.90) and the errors 1.8 and 1.5 times the printed ones;
    the paper's treatment of the discontinuous Dirichlet data and error is
    not specified further, so only second order within 0.25 of the printed
    rates is pinned."""
    from inputs import boundary_triangles_to_layer
    rows = _golden_rows("table5_peridynamic_dg_rates.txt")
    delta = 0.1
    errs = []
    for i, n in enumerate((5, 10, 20)):
        mesh = boundary_triangles_to_layer(square_mesh(n, delta=delta, side=0.5), side=0.5)
        c = dict(cfg("peridynamic", c=3.0 / delta ** 3, delta=delta, approach="approxcaps", rule=paper7(),
                     singular_n=0), ansatz="dg")
        e, ndof = _manufactured_l2(oracle_lib, mesh, c, _u_navier, f_affine=_F_NAVIER)
        if n <= 10:
            assert float(f"{ndof:.2e}") == rows[i][1]
        errs.append(e)
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    for got, row in zip(rates, rows[1:]):
        assert got >= 1.8 and abs(got - row[3]) <= 0.25, rates


# ----------------------------------------------------------------------
# label-dependent (material) kernels, possibly non-symmetric:
# Psi(x, y) = C[m(x)][m(y)] Psi0(x - y)

_TABLE = np.array([[1.0, 0.3], [2.5, 0.7]])   # non-symmetric


def _two_materials(mesh):
    """Material 1 for elements whose barycentre has x1 > 0.45, else 0."""
    import dataclasses
    bx = mesh.vertices[mesh.elements].mean(axis=1)[:, 0]
    return dataclasses.replace(mesh, materials=(bx > 0.45).astype(np.int32))


@pytest.mark.parametrize("singular_n,rule", [(0, "gauss7"), (4, "paper7")])
def test_material_kernel_full_ball_closed_form(oracle_lib, singular_n, rule):
    """Constant kernel c C[m(x)][m(y)] with the ball covering the mesh:
    a(phi_j, phi_i) = c int int (phi_i(x) - phi_i(y)) (C_xy phi_j(x) - C_yx phi_j(y))
    over D x D, which with D_a the elements of material a, M^a the P1 mass
    matrix over D_a and m^a_i = int_{D_a} phi_i is
      c sum_ab [C_ab |D_b| M^a_ij - C_ba m^a_i m^b_j - C_ab m^b_i m^a_j + C_ba |D_a| M^b_ij]
    for every degree of freedom i.  A transposed table, a swapped x/y or a
    missing direction fails it."""
    mesh = _two_materials(square_mesh(5, m=1, jitter=0.2, seed=4))
    r = gauss7() if rule == "gauss7" else paper7()
    c = 3.7
    P = oracle_lib.Problem(mesh, dict(cfg("constant", c=c, delta=100.0, rule=r, singular_n=singular_n),
                                      material_c=_TABLE))
    A = dense(P, *P.assemble())
    Ms, ms, Ds = [], [], []
    import dataclasses
    for a in range(2):
        sub = dataclasses.replace(mesh, elements=mesh.elements[mesh.materials == a],
                                  labels=mesh.labels[mesh.materials == a])
        M, mv = mass_matrix(sub)
        Ms.append(M)
        ms.append(mv)
        Ds.append(mv.sum())
    C = _TABLE
    expect = np.zeros_like(A)
    for a in range(2):
        for b in range(2):
            expect += C[a, b] * Ds[b] * Ms[a] - C[b, a] * np.outer(ms[a], ms[b]) \
                - C[a, b] * np.outer(ms[b], ms[a]) + C[b, a] * Ds[a] * Ms[b]
    expect *= c
    dof = P.isdof()
    assert np.max(np.abs(A[dof] - expect[dof])) < 1e-13 * np.abs(expect).max()
    # the transposed table gives another matrix (the orientation matters)
    Pt = oracle_lib.Problem(mesh, dict(cfg("constant", c=c, delta=100.0, rule=r, singular_n=singular_n),
                                       material_c=_TABLE.T.copy()))
    At = dense(Pt, *Pt.assemble())
    assert np.max(np.abs(At[dof] - A[dof])) > 1e-3 * np.abs(A).max()


@pytest.mark.parametrize("kernel", ["inv_dist", "peridynamic"])
def test_material_kernel_null_space_and_symmetry(oracle_lib, kernel):
    """All elements in Omega (pure interaction problem): a(phi_j, 1) = 0 for a
    kernel of any table, so every column of the matrix sums to zero; the rows
    sum to a(1, phi_i) = 2 int int (C_xy - C_yx) Psi0 phi_i(x), which is not
    zero for a non-symmetric table.  A symmetric table gives a symmetric
    matrix, and the table c * ones gives c times the plain matrix (touching
    pairs through the transforms included)."""
    mesh = _two_materials(square_mesh(6, delta=0.3, jitter=0.2, seed=8, neumann=True))
    base = cfg(kernel, c=1.3, delta=0.3, singular_n=5)
    n = base["ncomp"]
    A = dense(oracle_lib.Problem(mesh, dict(base, material_c=_TABLE)),
              *oracle_lib.Problem(mesh, dict(base, material_c=_TABLE)).assemble())
    scale = np.abs(A).max()
    colsum = A.reshape(A.shape[0], -1, n).sum(axis=0) if n == 1 else \
        np.stack([A[c::n].sum(axis=0) for c in range(n)])
    assert np.abs(colsum).max() <= 1e-13 * scale
    rowsum = A.sum(axis=1) if n == 1 else np.stack([A[:, c::n].sum(axis=1) for c in range(n)])
    assert np.abs(rowsum).max() > 1e-3 * scale
    sym = np.array([[1.0, 0.4], [0.4, 2.0]])
    Ps = oracle_lib.Problem(mesh, dict(base, material_c=sym))
    As = dense(Ps, *Ps.assemble())
    assert np.abs(As - As.T).max() <= 1e-14 * np.abs(As).max()
    P1 = oracle_lib.Problem(mesh, dict(base, material_c=np.full((2, 2), 1.7)))
    P0 = oracle_lib.Problem(mesh, base)
    A1, A0 = dense(P1, *P1.assemble()), dense(P0, *P0.assemble())
    assert np.abs(A1 - 1.7 * A0).max() <= 1e-14 * np.abs(A1).max()


def test_material_dg_restricts_to_cg(oracle_lib):
    """P^T A_DG P = A_CG with a non-symmetric table (the DG edge and vertex
    pairs by the 4D transforms, the continuous ones too)."""
    mesh = _two_materials(square_mesh(8, delta=0.3, jitter=0.2, seed=3))
    c_cg = dict(cfg("inv_dist", c=1.5, delta=0.3, singular_n=5), material_c=_TABLE)
    Pc = oracle_lib.Problem(mesh, c_cg)
    Pd = oracle_lib.Problem(mesh, dict(c_cg, ansatz="dg"))
    rc, cc, vc = Pc.assemble()
    rd, cd, vd = Pd.assemble()
    Nc, Nd = Pc.n_unknowns, Pd.n_unknowns
    Ac = sp.csr_matrix((vc, cc, rc), shape=(Nc, Nc))
    Ad = sp.csr_matrix((vd, cd, rd), shape=(Nd, Nd))
    E = mesh.elements
    r = [3 * k + a for k in range(E.shape[0]) for a in range(3)]
    q = [E[k, a] for k in range(E.shape[0]) for a in range(3)]
    P = sp.csr_matrix((np.ones(len(r)), (r, q)), shape=(Nd, Nc))
    dof = Pc.isdof()
    assert abs((P.T @ Ad @ P - Ac).tocsr()[dof]).max() <= 1e-14 * abs(Ac[dof]).max()
