"""The factorisation behind the mask form of the constant kernel (CPU only).

For a constant kernel and inclusion decided per outer point, the double
quadrature sums of a non-touching pair (Sec. 2.3, the four terms of the
bilinear form; Sec. 2.4.1, the product rule) factor into sums over one
element's rule.  The GPU row gather and diagonal sums evaluate the factored
form; these tests check, with random rules, determinants and status masks,
that it equals the plain double sums for both directions of a pair and for
the self pair.  Pure numpy; neither the oracle nor the GPU library is used.
"""
import numpy as np
import pytest


def _rule(rng, n):
    xi = rng.dirichlet(np.ones(3), size=n)          # barycentric points
    w = rng.uniform(0.05, 0.3, size=n)
    return w, xi                                      # phi_a(x_p) = xi[p, a]


def _double_sums(c, de, df, wo, po, wi, pi, s_e, s_f, self_pair):
    """X (3x3), De, Df (3x3) of the unordered pair by the plain double sums:
    direction (e, f) with the outer rule on e (points counted by s_e) and the
    inner rule on f, and, unless the pair is the self pair, direction (f, e)
    with the inner rule on e and the outer rule on f (counted by s_f)."""
    X = np.zeros((3, 3))
    De = np.zeros((3, 3))
    Df = np.zeros((3, 3))
    for p in range(len(wo)):
        for q in range(len(wi)):
            g = c * wo[p] * de * wi[q] * df * s_e[p]
            X -= g * np.outer(po[p], pi[q])
            De += g * np.outer(po[p], po[p])
            Df += g * np.outer(pi[q], pi[q])
    if not self_pair:
        for p in range(len(wi)):
            for q in range(len(wo)):
                g = c * wi[p] * de * wo[q] * df * s_f[q]
                X -= g * np.outer(pi[p], po[q])
                De += g * np.outer(pi[p], pi[p])
                Df += g * np.outer(po[q], po[q])
    return X, De, Df


def _factored(c, de, df, wo, po, wi, pi, m_e, m_f):
    """Row block of e against f and e's diagonal block from the one-element
    sums: M_O(m)_a = sum_p m_p w_p phi_a(x_p), T_O(m) = sum_p m_p w_p,
    Q_O(m) = sum_p m_p w_p phi phi^T, and the inner-rule sums over all points."""
    MO = lambda m: (m * wo) @ po
    TO = lambda m: float(np.sum(m * wo))
    QO = lambda m: np.einsum("p,pa,pb->ab", m * wo, po, po)
    MI, WI, QI = wi @ pi, float(np.sum(wi)), np.einsum("q,qa,qb->ab", wi, pi, pi)
    rows = -c * de * df * (np.outer(MO(m_e), MI) + np.outer(MI, MO(m_f)))
    diag = c * de * df * (QO(m_e) * WI + QI * TO(m_f))
    return rows, diag


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("P,Q", [(7, 7), (1, 7), (4, 7), (8, 3)])
def test_factored_blocks_equal_double_sums(seed, P, Q):
    rng = np.random.default_rng(1000 * seed + 10 * P + Q)
    wo, po = _rule(rng, P)
    wi, pi = (wo, po) if P == Q and seed % 2 == 0 else _rule(rng, Q)
    c = rng.uniform(0.5, 2.0)
    de, df = rng.uniform(0.1, 1.0, size=2)
    s_e = (rng.random(P) < 0.6).astype(float)
    s_f = (rng.random(P) < 0.6).astype(float)
    X, De, Df = _double_sums(c, de, df, wo, po, wi, pi, s_e, s_f, False)
    # e first: rows of e are the rows of X, e's diagonal block De
    rows_e, diag_e = _factored(c, de, df, wo, po, wi, pi, s_e, s_f)
    np.testing.assert_allclose(rows_e, X, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(diag_e, De, rtol=1e-12, atol=1e-14)
    # f's side: its rows are the columns of X, its diagonal block Df
    rows_f, diag_f = _factored(c, df, de, wo, po, wi, pi, s_f, s_e)
    np.testing.assert_allclose(rows_f, X.T, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(diag_f, Df, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_self_pair_takes_equal_masks(seed):
    """The self pair is integrated in one direction; its row block is
    X + X^T and its diagonal block De + Df, the factored form with me = mf."""
    rng = np.random.default_rng(77 + seed)
    wo, po = _rule(rng, 7)
    wi, pi = _rule(rng, 5)
    c, d = rng.uniform(0.5, 2.0), rng.uniform(0.1, 1.0)
    s = (rng.random(7) < 0.7).astype(float)
    X, De, Df = _double_sums(c, d, d, wo, po, wi, pi, s, np.zeros(7), True)
    rows, diag = _factored(c, d, d, wo, po, wi, pi, s, s)
    np.testing.assert_allclose(rows, X + X.T, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(diag, De + Df, rtol=1e-12, atol=1e-14)


def test_a_dropped_term_is_caught():
    """Leaving out the second direction's term of the rows must fail the check."""
    rng = np.random.default_rng(5)
    wo, po = _rule(rng, 7)
    s_e = (rng.random(7) < 0.5).astype(float)
    s_f = (rng.random(7) < 0.5).astype(float)
    X, _, _ = _double_sums(1.0, 0.5, 0.7, wo, po, wo, po, s_e, s_f, False)
    MO = (s_e * wo) @ po
    MI = wo @ po
    wrong = -1.0 * 0.5 * 0.7 * np.outer(MO, MI)
    assert not np.allclose(wrong, X, rtol=1e-6)
