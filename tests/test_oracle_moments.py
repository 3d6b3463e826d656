"""Pins of the oracle's moment operator (Section 2, Eqs. 1moment/2moment).

* brute force: M2 formed by enumerating ordered pairs of distinct tokens (or
  distinct leaves) of every sample, then applied to S, against the implicit
  operator O = M2 S (which uses c c^T - diag(c));
* Monte Carlo: the empirical M2 of sampled documents with alpha0 > 0
  approaches sum_i ahat_i mu_i mu_i^T (Lemma topic), which fails if a
  length weight or the alpha0 correction is wrong.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from planted import exact_m2, planted_topics


def _tokens_of(C):
    """Token list of every row of a count CSR (expand counts)."""
    Cs = C.to_scipy(np.float64)
    out = []
    for t in range(Cs.shape[0]):
        row = Cs.getrow(t)
        toks = []
        for w, c in zip(row.indices, row.data):
            toks += [int(w)] * int(round(c))
        out.append(toks)
    return out


def _brute_m2_docs(tokens, d, alpha0):
    n = len(tokens)
    M1 = np.zeros(d)
    pairs = np.zeros((d, d))
    for toks in tokens:
        l = len(toks)
        for w in toks:
            M1[w] += 1.0 / l / n
        for p in range(l):
            for q in range(l):
                if p != q:
                    pairs[toks[p], toks[q]] += 1.0 / (l * (l - 1))
    return (alpha0 + 1.0) / n * pairs - alpha0 * np.outer(M1, M1)


@pytest.mark.parametrize("alpha0", [0.0, 0.7, 2.0])
def test_m2_apply_matches_token_pair_enumeration(alpha0):
    inst = synth.lda(d=9, k=3, alpha0=1.0, beta=0.5, n_docs=40, mean_len=7.0, seed=11)
    S = synth.projection(9, 6, seed=3)
    M2 = _brute_m2_docs(_tokens_of(inst.C), 9, alpha0)
    O = oracle.m2_apply(inst.C, S, alpha0, normalize=True)
    np.testing.assert_allclose(O, M2 @ S, rtol=0, atol=1e-13 * np.abs(M2 @ S).max())


@pytest.mark.parametrize("alpha0", [0.0, 0.1, 0.5])
def test_m2_apply_graph_matches_leaf_pair_enumeration(alpha0):
    inst = synth.mmsb(n=60, k=3, alpha0=0.5, p=0.6, q=0.1, n_x=30, seed=5)
    Cs = inst.C.to_scipy(np.float64).toarray()
    n, d = Cs.shape
    M1 = Cs.mean(axis=0)
    pairs = np.zeros((d, d))
    for x in range(n):
        leaves = np.nonzero(Cs[x])[0]
        for a in leaves:
            for b in leaves:
                if a != b:
                    pairs[a, b] += 1.0
    M2 = (alpha0 + 1.0) / n * pairs - alpha0 * np.outer(M1, M1)
    S = synth.projection(d, 5, seed=4)
    O = oracle.m2_apply(inst.C, S, alpha0, normalize=False)
    np.testing.assert_allclose(O, M2 @ S, rtol=0, atol=1e-13 * max(1.0, np.abs(M2 @ S).max()))


def test_first_moment_definition():
    inst = synth.lda(d=7, k=2, alpha0=1.0, beta=0.5, n_docs=25, mean_len=6.0, seed=2)
    toks = _tokens_of(inst.C)
    M1 = np.zeros(7)
    for tk in toks:
        for w in tk:
            M1[w] += 1.0 / len(tk) / len(toks)
    np.testing.assert_allclose(oracle.first_moment(inst.C, True), M1, atol=1e-15)
    assert abs(M1.sum() - 1.0) < 1e-12


@pytest.mark.slow
def test_m2_expectation_matches_topic_lemma():
    """Monte Carlo: E[M2] = sum_i ahat_i mu_i mu_i^T (Lemma topic) at alpha0 = 1."""
    d, k = 6, 3
    mu, _ = planted_topics(d, k, seed=21, beta=0.8)
    alpha0 = 1.0
    inst = synth.lda(d=d, k=k, alpha0=alpha0, beta=1.0, n_docs=200000, mean_len=8.0, seed=22, mu=mu)
    ahat = np.full(k, 1.0 / k)
    exact = exact_m2(mu, ahat)
    O = oracle.m2_apply(inst.C, np.eye(d), alpha0, normalize=True)
    err = np.abs(O - exact).max()
    assert err < 1.5e-2 * np.abs(exact).max(), err
    # dropping the alpha0 correction of Eq. 2moment_topic is visibly wrong
    M1 = oracle.first_moment(inst.C, True)
    assert np.abs(O + alpha0 * np.outer(M1, M1) - exact).max() > 20 * err
