"""Statistics and determinism of the seeded input generators."""
import numpy as np

import synth


def test_mmsb_degree_and_structure():
    g = synth.mmsb(n=2000, k=5, alpha0=0.5, p=0.3, q=0.02, n_x=1000, seed=3)
    # undirected, no self loops; expected edge probability q + (p - q) E<pi_i, pi_j>
    pi = g.pi
    s = (pi.sum(0) ** 2 - (pi ** 2).sum(0)).sum() / (len(pi) * (len(pi) - 1))
    exp_edges = (g.meta["q"] + (g.meta["p"] - g.meta["q"]) * s) * len(pi) * (len(pi) - 1) / 2
    assert abs(g.n_edges - exp_edges) < 5 * np.sqrt(exp_edges)
    assert g.C.n_rows == 1000 and g.C.n_cols == 1000 and g.C.vals is None
    assert np.all(np.diff(g.C.rowptr) >= 0)
    # C^T is the transpose
    np.testing.assert_array_equal(g.CT.to_scipy().toarray(), g.C.to_scipy().toarray().T)
    np.testing.assert_allclose(pi.sum(1), 1.0, atol=1e-12)


def test_mmsb_deterministic():
    a = synth.mmsb(n=300, k=3, alpha0=0.3, p=0.4, q=0.05, seed=9)
    b = synth.mmsb(n=300, k=3, alpha0=0.3, p=0.4, q=0.05, seed=9)
    np.testing.assert_array_equal(a.C.colidx, b.C.colidx)
    np.testing.assert_array_equal(a.C.rowptr, b.C.rowptr)


def test_lda_lengths_views_and_topics():
    inst = synth.lda(d=500, k=4, alpha0=1.0, beta=0.1, n_docs=3000, mean_len=50.0, seed=5)
    assert inst.lengths.min() >= 3
    assert abs(inst.lengths.mean() - 50.0) < 1.0
    full = inst.C.to_scipy().toarray()
    np.testing.assert_array_equal(full.sum(1), inst.lengths)
    parts = sum(v.to_scipy().toarray() for v in inst.views)
    np.testing.assert_array_equal(parts, full)
    for v in inst.views:
        assert np.asarray(v.to_scipy().sum(1)).min() >= 1
    np.testing.assert_allclose(inst.mu.sum(0), 1.0, atol=1e-12)
    # word frequencies follow mu @ E[h]
    freq = full.sum(0) / full.sum()
    expect = inst.mu @ inst.h.mean(0)
    assert np.abs(freq - expect).max() < 0.01


def test_initial_factors_orthonormal_and_permutations():
    P = synth.initial_factors(7, seed=1, restart=2)
    np.testing.assert_allclose(P.T @ P, np.eye(7), atol=1e-12)
    assert not np.allclose(P, synth.initial_factors(7, seed=1, restart=3))
    perms = synth.permutations(11, 4, seed=2)
    assert perms.shape == (4, 11) and perms.dtype == np.int32
    for p in perms:
        np.testing.assert_array_equal(np.sort(p), np.arange(11))


def test_poisson_graph_counts_have_the_model_mean_and_variance():
    """Section 2.2 Poisson model: over the X x A pairs the counts have mean
    lambda = pi_i^T P pi_j and (Poisson) variance equal to the mean, within
    sampling error; pairs of very different lambda are checked by bins."""
    g = synth.mmsb_weighted(3000, 4, 0.4, 0.6, 0.05, seed=9)
    lam = (g.pi[g.X] @ g.P @ g.pi[g.A].T).ravel()
    G = g.C.to_scipy(np.float64).toarray().ravel()
    for lo, hi in ((0.0, 0.1), (0.1, 0.3), (0.3, 0.7)):
        m = (lam >= lo) & (lam < hi)
        if m.sum() < 20000:
            continue
        mean, var = G[m].mean(), G[m].var()
        se = np.sqrt(lam[m].mean() / m.sum())
        assert abs(mean - lam[m].mean()) < 5 * se
        assert abs(var - mean) < 0.05 * mean + 5 * se
    assert g.C.vals.max() >= 2.0                        # counts, not indicators


def test_bipartite_graph_has_edges_only_across_and_the_model_rate():
    b = synth.bipartite(1500, 1000, 3, 0.5, 0.5, 0.05, poisson=False, seed=4)
    assert b.C.n_rows == 1500 and b.C.n_cols == 1000
    lam = b.pi_u @ b.P @ b.pi_v.T
    assert abs(b.C.nnz - lam.sum()) < 5 * np.sqrt(lam.sum())
    np.testing.assert_array_equal(b.CT.to_scipy().toarray(), b.C.to_scipy().toarray().T)
    bw = synth.bipartite(1500, 1000, 3, 0.5, 0.5, 0.05, poisson=True, seed=4)
    assert abs(bw.C.vals.sum() - lam.sum()) < 5 * np.sqrt(lam.sum())


def test_generalised_sampler_reproduces_the_bernoulli_graph():
    """The generalised sampler in Bernoulli mode draws the same random numbers
    as the undirected sampler, so it returns the same edge set."""
    n, k, seed = 2000, 5, 3
    pi = synth.rng(seed, synth.S_PI).dirichlet(np.full(k, 0.1), size=n)
    src, dst = synth._mmsb_edges(n, pi, 0.3, 0.05, seed, 1e-15)
    eseed = int(synth.rng(seed, synth.S_EDGES).integers(0, 2**63 - 1))
    s2, d2, w2 = synth._pairs_general(pi, pi, True, False, 0.3, 0.05, eseed, 1e-15)
    np.testing.assert_array_equal(src, s2)
    np.testing.assert_array_equal(dst, d2)
    assert np.all(w2 == 1.0)
