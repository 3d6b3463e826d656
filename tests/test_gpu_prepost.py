"""GPU parity of the FP64 pre- and post-processing (M2 operator, randomized
whitener, topic unwhitening, membership recovery) and of the measurement-only
tensor/residual, against the FP64 oracle.

Bars: FP64 stages within 1e-11 relative (M2 operator), 1e-9 relative on W
after the sign rule (eigenvector conditioning), 1e-9 on mu; memberships
(FP32 output of FP64 arithmetic) within 1e-6 absolute except where the oracle's
value lies within 1e-6 of the threshold tau; explicit tensor within 1e-12
relative and residuals within 1e-9 relative."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import csr_dev, dev, f32_round, host, padded, phi_rows, rel, to_dev
from planted import exact_m2, planted_topics, planted_whitened_factors

from paper_1309_0787_amd import otm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("alpha0", [0.0, 1.0])
def test_m2_apply_documents(alpha0):
    inst = synth.lda(d=800, k=5, alpha0=1.0, beta=0.1, n_docs=1500, mean_len=30.0, seed=2)
    S = synth.projection(800, 12, seed=3)
    O = otm.m2_apply(csr_dev(inst.C), csr_dev(inst.CT), True, alpha0, to_dev(S, torch.float64))
    torch.cuda.synchronize()
    ref = oracle.m2_apply(inst.C, S, alpha0, normalize=True)
    assert rel(host(O), ref) < 1e-11


def test_m2_apply_graph():
    g = synth.make("mmsb_small")
    S = synth.projection(g.C.n_cols, 20, seed=1)
    O = otm.m2_apply(csr_dev(g.C), csr_dev(g.CT), False, 0.1, to_dev(S, torch.float64))
    torch.cuda.synchronize()
    assert rel(host(O), oracle.m2_apply(g.C, S, 0.1, normalize=False)) < 1e-11


def test_m2_apply_rejects_short_documents():
    C = synth.CSR(2, 3, np.array([0, 2, 3], dtype=np.int32), np.array([0, 1, 2], dtype=np.int32),
                  np.array([1, 1, 1], dtype=np.float32))     # second document has one token
    with pytest.raises(otm.OtmError):
        otm.m2_apply(csr_dev(C), csr_dev(C.transpose()), True, 1.0, to_dev(np.ones((3, 2)), torch.float64))


@pytest.mark.parametrize("d,k,kt", [(30, 4, 8), (500, 10, 20), (2000, 50, 100), (3000, 100, 200), (400, 128, 256)])
def test_whitener_exact_rank_k(d, k, kt):
    mu, ahat = planted_topics(d, k, seed=d + k)
    M2 = exact_m2(mu, ahat)
    S = synth.projection(d, kt, seed=7)
    O = M2 @ S
    W, ev, Wlo = otm.whitener(to_dev(O, torch.float64), to_dev(S, torch.float64), k, w_lo_dtype=otm.BF16)
    torch.cuda.synchronize()
    Wg = host(W)
    Wref, evref = oracle.whitener_rsvd(O, S, k)
    np.testing.assert_allclose(Wg.T @ M2 @ Wg, np.eye(k), atol=1e-10)
    assert rel(Wg, Wref) < 1e-9
    np.testing.assert_allclose(host(ev), evref, rtol=1e-10)
    np.testing.assert_array_equal(host(Wlo), torch.as_tensor(Wg).to(torch.bfloat16).double().numpy())
    ld = Wlo.stride(0)                              # the row-padded buffer behind the view: zeros in the padding
    assert ld == otm.default_ldw(k, otm.BF16)
    assert np.all(host(Wlo.as_strided((d, ld), (ld, 1)))[:, k:] == 0.0)


def test_whitener_sampled_graph():
    """Same (O, Q) on both sides: the oracle's power-iterated sketch (q = 3)."""
    g = synth.make("mmsb_small")
    S = synth.projection(g.C.n_cols, 20, seed=1)
    Q, O = oracle.power_sketch(g.C, S, 0.1, False, 3)
    W, ev, Wlo = otm.whitener(to_dev(O, torch.float64), to_dev(Q, torch.float64), 10, w_lo_dtype=otm.F32)
    torch.cuda.synchronize()
    Wref, evref = oracle.whitener_rsvd(O, Q, 10)
    assert rel(host(W), Wref) < 1e-9
    np.testing.assert_allclose(host(ev), evref, rtol=1e-10)
    np.testing.assert_array_equal(host(Wlo), f32_round(host(W)))
    _, _, Wlo2 = otm.whitener(to_dev(O, torch.float64), to_dev(Q, torch.float64), 10, w_lo_dtype=otm.F32, ldw_lo=13)
    torch.cuda.synchronize()
    assert Wlo2.stride(0) == 13
    np.testing.assert_array_equal(host(Wlo2), host(Wlo))
    assert np.all(host(Wlo2.as_strided((Wlo2.shape[0], 13), (13, 1)))[:, 10:] == 0.0)


@pytest.mark.parametrize("normalize", [False, True])
def test_power_sketch_chain(normalize):
    """GPU sketch (Cholesky-QR bases) and oracle sketch (Householder QR bases)
    span the same spaces, so the whiteners agree after the sign rule."""
    if normalize:
        inst = synth.lda(d=1500, k=6, alpha0=1.0, beta=0.1, n_docs=3000, mean_len=50.0, seed=3)
        C, CT, a0, k = inst.C, inst.CT, 1.0, 6
    else:
        inst = synth.make("mmsb_small")
        C, CT, a0, k = inst.C, inst.CT, 0.1, 10
    S = synth.projection(C.n_cols, 2 * k, seed=4)
    Qg, Og = otm.power_sketch(csr_dev(C), csr_dev(CT), normalize, a0, to_dev(S, torch.float64), 3)
    W, ev, _ = otm.whitener(Og, Qg, k)
    torch.cuda.synchronize()
    Qh = host(Qg)
    # orthonormal to about eps * cond(Y) after the second Cholesky-QR pass; only
    # span(Q) matters downstream, which the whitener comparison below checks
    np.testing.assert_allclose(Qh.T @ Qh, np.eye(2 * k), atol=1e-10)
    Qo, Oo = oracle.power_sketch(C, S, a0, normalize, 3)
    Wref, evref = oracle.whitener_rsvd(Oo, Qo, k)
    assert rel(host(W), Wref) < 1e-8
    np.testing.assert_allclose(host(ev), evref, rtol=1e-9)


@pytest.mark.parametrize("d,m", [(50, 1), (300, 7), (400, 13), (500, 37), (1000, 64), (3000, 100), (5000, 200),
                                 (2000, 256)])
def test_orthonormalize(d, m):
    """m <= 200: Cholesky QR gives the QR factor whose R has a positive
    diagonal, which is unique, so it must equal NumPy's QR after that sign fix.
    m > 200: Y (Y^T Y)^(-1/2); orthonormal with the same span."""
    gen = np.random.default_rng(d + m)
    Y = gen.standard_normal((d, m)) @ np.diag(np.logspace(0, 3, m))     # cond(Y) = 1e3
    Q = host(otm.orthonormalize(to_dev(Y, torch.float64)))
    np.testing.assert_allclose(Q.T @ Q, np.eye(m), atol=1e-12)
    if m <= 200:
        Qr, R = np.linalg.qr(Y)
        Qr = Qr * np.sign(np.diag(R))
        assert rel(Q, Qr) < 1e-11
    else:
        assert rel(Q @ (Q.T @ Y), Y) < 1e-12


def test_orthonormalize_rank_deficient():
    gen = np.random.default_rng(1)
    Y = gen.standard_normal((400, 10))
    Y[:, 7] = Y[:, 2] - 0.5 * Y[:, 4]
    with pytest.raises(otm.OtmError):
        otm.orthonormalize(to_dev(Y, torch.float64))


def test_whitener_not_psd():
    g = np.random.default_rng(0)
    A = g.standard_normal((40, 40))
    S = synth.projection(40, 8, seed=1)
    O = -(A @ A.T) @ S
    with pytest.raises(otm.OtmNotPSD):
        otm.whitener(to_dev(O, torch.float64), to_dev(S, torch.float64), 4)


def test_unwhiten_topics_exact_and_vs_oracle():
    d, k = 600, 12
    mu, ahat = planted_topics(d, k, seed=5)
    S = synth.projection(d, 2 * k, seed=2)
    Wref, _ = oracle.whitener_rsvd(exact_m2(mu, ahat) @ S, S, k)
    _, lam, Phi = planted_whitened_factors(Wref, mu, ahat)
    Phi32 = f32_round(Phi)
    mu_g, ah_g, lam_g = otm.unwhiten_topics(to_dev(Wref, torch.float64), phi_rows(Phi32))
    torch.cuda.synchronize()
    mu_o, ah_o, lam_o = oracle.unwhiten_topics(Wref, Phi32)
    assert rel(host(mu_g), mu_o) < 1e-9
    np.testing.assert_allclose(host(ah_g), ah_o, rtol=1e-10)
    np.testing.assert_allclose(host(lam_g), lam_o, rtol=1e-10)
    assert np.abs(host(mu_g) - mu).max() < 1e-5        # FP32 factors: exact up to their rounding


@pytest.mark.parametrize("tau", [0.0, 0.1])
@pytest.mark.parametrize("ydt", [otm.F32, otm.BF16])
def test_recover_pi_vs_oracle(tau, ydt):
    n, k = 1037, 24
    gen = np.random.default_rng(4)
    Y = gen.standard_normal((n, k))
    Phi = f32_round(synth.initial_factors(k, seed=2) * 1.5 + 0.05 * gen.standard_normal((k, k)))
    tdt = torch.bfloat16 if ydt == otm.BF16 else torch.float32
    Yd = padded(Y, otm.default_ldy(k), tdt)
    Yh = host(Yd)[:, :k]
    Pi = otm.recover_pi(Yd, k, phi_rows(Phi), tau=tau)
    torch.cuda.synchronize()
    ref = oracle.recover_pi(Yh, Phi, tau)
    got = host(Pi)
    near = np.zeros_like(ref, dtype=bool)
    if tau > 0:
        raw = oracle.recover_pi(Yh, Phi, 0.0)
        near = np.abs(raw - tau) < 1e-6
        cols = near.any(axis=0)
        near[:, cols] = True
    assert np.abs(got - ref)[~near].max() < 1e-6


def test_tensor_form_and_residual():
    n, k = 333, 9
    gen = np.random.default_rng(8)
    YA, YB, YC = (gen.standard_normal((n, k)) for _ in range(3))
    ybar = np.stack([YA.mean(0), YB.mean(0), YC.mean(0)])
    YA, YB, YC, ybar = (f32_round(x) for x in (YA, YB, YC, ybar))
    ldy = otm.default_ldy(k)
    T = otm.tensor_form(padded(YA, ldy, torch.float32), padded(YB, ldy, torch.float32),
                        padded(YC, ldy, torch.float32), k, to_dev(ybar), 0.8)
    torch.cuda.synchronize()
    Tref = oracle.whitened_tensor(YA, YB, YC, ybar, 0.8)
    assert rel(host(T), Tref) < 1e-12
    Phis = np.stack([f32_round(synth.initial_factors(k, seed=s)) for s in range(3)])
    R = otm.residual(T, torch.stack([phi_rows(P) for P in Phis]))
    torch.cuda.synchronize()
    Rref = np.array([oracle.residual(Tref, P) for P in Phis])
    np.testing.assert_allclose(host(R), Rref, rtol=1e-9)
