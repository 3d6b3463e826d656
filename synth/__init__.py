"""Seeded synthetic inputs for the online tensor method (MMSB graphs, LDA corpora).

Input generation only.  This module holds none of the method's arithmetic:
no moments, no whitening, no tensor products.  Both the FP64 oracle and the
GPU path consume what it produces, and nothing else is shared between them.

Every random draw comes from an independent Philox stream keyed by
(seed, stream id), so each piece (memberships, edges, partition, topics,
lengths, tokens, projection, initial factors, permutations) can be
regenerated on its own.

Models (Section 2):
* MMSB (Section 2.2): pi_u ~ Dir(alpha), undirected G_ij ~ Ber(pi_i^T P pi_j),
  with P = q 1 1^T + (p - q) I.  No self-loops.  Nodes are split at random
  into a sample set X and a leaf set A; the observed matrix is G[X, A].
* LDA (Section 2.1): topics mu_j ~ Dir(beta 1_d), document mixtures
  h ~ Dir(alpha), lengths l ~ Poisson(mean_len) redrawn while l < 3,
  tokens iid given h.  Token positions are dealt round-robin into three
  views A, B, C (position mod 3), so each view holds at least one token and
  the views are independent given h.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 13090787

# Stream ids (one independent Philox stream each).
S_PI, S_EDGES, S_PARTITION, S_TOPICS, S_MIX, S_LENGTHS, S_TOKENS, S_WORDS, \
    S_PROJ, S_PHI0, S_PERM, S_MISC = range(12)

_HERE = os.path.dirname(os.path.abspath(__file__))
_PAIRS_SRC = os.path.join(_HERE, "mmsb_pairs.c")
_PAIRS_SO = os.path.join(_HERE, "_mmsb_pairs.so")


def rng(seed: int, stream: int, sub: int = 0) -> np.random.Generator:
    """Independent Philox generator for (seed, stream, sub)."""
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, stream, sub])))


# --------------------------------------------------------------------------
# CSR container
# --------------------------------------------------------------------------
@dataclass
class CSR:
    """Compressed sparse rows: int32 rowptr/colidx, float32 values or None (all ones)."""
    n_rows: int
    n_cols: int
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def values_or_ones(self) -> np.ndarray:
        if self.vals is None:
            return np.ones(self.nnz, dtype=np.float32)
        return self.vals

    def to_scipy(self, dtype=np.float64):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values_or_ones().astype(dtype), self.colidx, self.rowptr),
                             shape=(self.n_rows, self.n_cols))

    @staticmethod
    def from_scipy(m, implicit_ones: bool = False) -> "CSR":
        m = m.tocsr()
        m.sort_indices()
        m.sum_duplicates()
        vals = None if implicit_ones else np.asarray(m.data, dtype=np.float32)
        return CSR(m.shape[0], m.shape[1], np.asarray(m.indptr, dtype=np.int32),
                   np.asarray(m.indices, dtype=np.int32), vals)

    def transpose(self) -> "CSR":
        t = self.to_scipy(np.float32).T.tocsr()
        return CSR.from_scipy(t, implicit_ones=self.vals is None)

    def row_slice(self, r0: int, r1: int) -> "CSR":
        p0, p1 = int(self.rowptr[r0]), int(self.rowptr[r1])
        vals = None if self.vals is None else self.vals[p0:p1].copy()
        return CSR(r1 - r0, self.n_cols, (self.rowptr[r0:r1 + 1] - p0).astype(np.int32),
                   self.colidx[p0:p1].copy(), vals)


# --------------------------------------------------------------------------
# MMSB
# --------------------------------------------------------------------------
def _pairs_lib():
    if not os.path.exists(_PAIRS_SO) or os.path.getmtime(_PAIRS_SO) < os.path.getmtime(_PAIRS_SRC):
        build_pairs()
    lib = ctypes.CDLL(_PAIRS_SO)
    p = ctypes.c_void_p
    lib.mmsb_count.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, p, p, p, p]
    lib.mmsb_fill.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, p, p, p, p, p]
    g = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
         ctypes.c_uint64, p, p, p, p, p, p]
    lib.pairs_count.argtypes = g + [p]
    lib.pairs_fill.argtypes = g + [p, p, p]
    return lib


def build_pairs() -> None:
    """Compile the edge sampler (plain C, OpenMP)."""
    tmp = _PAIRS_SO + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _PAIRS_SRC, "-lm"])
    os.replace(tmp, _PAIRS_SO)


@dataclass
class MMSBInstance:
    n: int
    k: int
    alpha: np.ndarray          # (k,) Dirichlet parameters
    P: np.ndarray              # (k, k) block matrix
    pi: np.ndarray             # (n, k) memberships, rows on the simplex
    X: np.ndarray              # sample node ids (sorted)
    A: np.ndarray              # leaf node ids (sorted)
    C: CSR                     # G[X, A], implicit ones
    CT: CSR                    # G[A, X] = C^T, implicit ones
    n_edges: int = 0
    meta: dict = field(default_factory=dict)


def _mmsb_edges(n: int, pi: np.ndarray, p: float, q: float, seed: int, pi_floor: float):
    """Undirected edge list (src < dst) of the Bernoulli MMSB with
    P = q 1 1^T + (p - q) I, sampled by the C helper."""
    mask = pi >= pi_floor
    pptr = np.zeros(n + 1, dtype=np.int64)
    pptr[1:] = np.cumsum(mask.sum(1))
    rows, cols = np.nonzero(mask)
    pidx = cols.astype(np.int32)
    pval = pi[rows, cols].astype(np.float64)
    lib = _pairs_lib()
    eseed = int(rng(seed, S_EDGES).integers(0, 2**63 - 1))
    counts = np.zeros(n, dtype=np.int64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    lib.mmsb_count(n, p, q, eseed, ptr(pptr), ptr(pidx), ptr(pval), ptr(counts))
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    upper = np.zeros(int(offsets[-1]), dtype=np.int32)
    lib.mmsb_fill(n, p, q, eseed, ptr(pptr), ptr(pidx), ptr(pval), ptr(offsets), ptr(upper))
    src = np.repeat(np.arange(n, dtype=np.int64), counts)
    return src, upper.astype(np.int64)


def _sparse_memberships(pi: np.ndarray, pi_floor: float):
    mask = pi >= pi_floor
    ptr = np.zeros(pi.shape[0] + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(mask.sum(1))
    rows, cols = np.nonzero(mask)
    return ptr, cols.astype(np.int32), pi[rows, cols].astype(np.float64)


def _pairs_general(pi_rows: np.ndarray, pi_cols: np.ndarray, triangular: bool, poisson: bool, p: float, q: float,
                   eseed: int, pi_floor: float):
    """Edges (row index, column index, weight) between two node sets (or
    within one set, j > i, when triangular) under the Bernoulli or Poisson
    model with P = q 1 1^T + (p - q) I, sampled by the C helper."""
    lib = _pairs_lib()
    rp, ri, rv = _sparse_memberships(pi_rows, pi_floor)
    cp, ci, cv = _sparse_memberships(pi_cols, pi_floor)
    nr, nc = pi_rows.shape[0], pi_cols.shape[0]
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    counts = np.zeros(nr, dtype=np.int64)
    args = (nr, nc, int(triangular), int(poisson), p, q, eseed, ptr(rp), ptr(ri), ptr(rv), ptr(cp), ptr(ci), ptr(cv))
    lib.pairs_count(*args, ptr(counts))
    offsets = np.zeros(nr + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    cols = np.zeros(int(offsets[-1]), dtype=np.int32)
    w = np.zeros(int(offsets[-1]), dtype=np.float32)
    lib.pairs_fill(*args, ptr(offsets), ptr(cols), ptr(w))
    src = np.repeat(np.arange(nr, dtype=np.int64), counts)
    return src, cols.astype(np.int64), w


def graph_block(src: np.ndarray, dst: np.ndarray, n: int, rows: np.ndarray, cols: np.ndarray,
                weights: np.ndarray | None = None) -> CSR:
    """G[rows, cols] of the undirected graph with edges (src, dst) (both
    directions), rows and cols sorted node ids; implicit ones unless weights."""
    import scipy.sparse as sp
    pos_r = np.full(n, -1, dtype=np.int64)
    pos_r[rows] = np.arange(len(rows))
    pos_c = np.full(n, -1, dtype=np.int64)
    pos_c[cols] = np.arange(len(cols))
    r = np.concatenate([src, dst])
    c = np.concatenate([dst, src])
    keep = (pos_r[r] >= 0) & (pos_c[c] >= 0)
    w = np.ones(int(keep.sum()), dtype=np.float32) if weights is None else \
        np.concatenate([weights, weights]).astype(np.float32)[keep]
    m = sp.csr_matrix((w, (pos_r[r[keep]], pos_c[c[keep]])), shape=(len(rows), len(cols)))
    return CSR.from_scipy(m, implicit_ones=weights is None)


def mmsb(n: int, k: int, alpha0: float, p: float, q: float, n_x: int | None = None,
         seed: int = BASE_SEED, pi_floor: float = 1e-15) -> MMSBInstance:
    """Draw an MMSB graph and its X/A split.

    pi_floor: membership entries below it are dropped from the edge
    probabilities (each dropped term changes a probability by < pi_floor).
    """
    alpha = np.full(k, alpha0 / k)
    pi = rng(seed, S_PI).dirichlet(alpha, size=n)
    P = np.full((k, k), q) + (p - q) * np.eye(k)
    src, dst = _mmsb_edges(n, pi, p, q, seed, pi_floor)
    # split nodes
    n_x = n // 2 if n_x is None else n_x
    perm = rng(seed, S_PARTITION).permutation(n)
    X = np.sort(perm[:n_x])
    A = np.sort(perm[n_x:])
    C = graph_block(src, dst, n, X, A)
    return MMSBInstance(n=n, k=k, alpha=alpha, P=P, pi=pi, X=X, A=A, C=C, CT=C.transpose(),
                        n_edges=int(len(src)), meta=dict(alpha0=alpha0, p=p, q=q, seed=seed))


@dataclass
class MMSBFour:
    """An MMSB graph with its nodes split into the sample set X and the three
    leaf sets A, B, C of Section 2.2.  blocks[(R, S)] = G[R, S] (CSR) for the
    pairs the method reads: (X,A), (X,B), (X,C), their transposes, and
    (B,A), (C,A) for the memberships of the B and C nodes."""
    n: int
    k: int
    alpha: np.ndarray
    P: np.ndarray
    pi: np.ndarray
    sets: dict                 # name -> sorted node ids
    blocks: dict
    n_edges: int = 0
    meta: dict = field(default_factory=dict)


FOUR_BLOCKS = (("X", "A"), ("X", "B"), ("X", "C"), ("A", "X"), ("B", "X"), ("C", "X"), ("B", "A"), ("C", "A"),
               ("A", "B"), ("A", "C"))


def mmsb_four(n: int, k: int, alpha0: float, p: float, q: float, fractions=(0.25, 0.25, 0.25, 0.25),
              seed: int = BASE_SEED, pi_floor: float = 1e-15, poisson: bool = False) -> MMSBFour:
    """The same Bernoulli MMSB as mmsb() (same memberships and edges for the
    same seed), or the Poisson model's counts (as mmsb_weighted()), with the
    nodes split at random into X, A, B, C of the given fractions (Section 2.2)."""
    alpha = np.full(k, alpha0 / k)
    pi = rng(seed, S_PI).dirichlet(alpha, size=n)
    P = np.full((k, k), q) + (p - q) * np.eye(k)
    w = None
    if poisson:
        eseed = int(rng(seed, S_EDGES, 1).integers(0, 2**63 - 1))
        src, dst, w = _pairs_general(pi, pi, True, True, p, q, eseed, pi_floor)
    else:
        src, dst = _mmsb_edges(n, pi, p, q, seed, pi_floor)
    perm = rng(seed, S_PARTITION, 4).permutation(n)
    sizes = [int(round(f * n)) for f in fractions[:3]]
    cuts = np.cumsum([0] + sizes + [n - sum(sizes)])
    sets = {name: np.sort(perm[cuts[i]:cuts[i + 1]]) for i, name in enumerate("XABC")}
    blocks = {(r, c): graph_block(src, dst, n, sets[r], sets[c], weights=w) for r, c in FOUR_BLOCKS}
    return MMSBFour(n=n, k=k, alpha=alpha, P=P, pi=pi, sets=sets, blocks=blocks, n_edges=int(len(src)),
                    meta=dict(alpha0=alpha0, p=p, q=q, seed=seed, model="poisson" if poisson else "bernoulli"))


def mmsb_weighted(n: int, k: int, alpha0: float, p: float, q: float, n_x: int | None = None,
                  seed: int = BASE_SEED, pi_floor: float = 1e-15) -> MMSBInstance:
    """The Poisson model of Section 2.2 (weighted edges): undirected counts
    G_ij ~ Poisson(pi_i^T P pi_j), P = q 1 1^T + (p - q) I, no self-loops; the
    observed G[X, A] carries the counts as values."""
    alpha = np.full(k, alpha0 / k)
    pi = rng(seed, S_PI).dirichlet(alpha, size=n)
    P = np.full((k, k), q) + (p - q) * np.eye(k)
    eseed = int(rng(seed, S_EDGES, 1).integers(0, 2**63 - 1))
    src, dst, w = _pairs_general(pi, pi, True, True, p, q, eseed, pi_floor)
    n_x = n // 2 if n_x is None else n_x
    perm = rng(seed, S_PARTITION).permutation(n)
    X = np.sort(perm[:n_x])
    A = np.sort(perm[n_x:])
    C = graph_block(src, dst, n, X, A, weights=w)
    return MMSBInstance(n=n, k=k, alpha=alpha, P=P, pi=pi, X=X, A=A, C=C, CT=C.transpose(), n_edges=int(len(src)),
                        meta=dict(alpha0=alpha0, p=p, q=q, seed=seed, model="poisson"))


@dataclass
class BipartiteInstance:
    """A bipartite graph between node sets U (rows) and V (columns), both with
    Dirichlet memberships over the same k communities (the business-user
    setting of Section 6): C = G[U, V], CT = G[V, U]."""
    k: int
    alpha: np.ndarray
    P: np.ndarray
    pi_u: np.ndarray
    pi_v: np.ndarray
    C: CSR
    CT: CSR
    meta: dict = field(default_factory=dict)


def bipartite(n_u: int, n_v: int, k: int, alpha0: float, p: float, q: float, poisson: bool = True,
              seed: int = BASE_SEED, pi_floor: float = 1e-15) -> BipartiteInstance:
    """G[u, v] ~ Poisson (or Bernoulli) of pi_u^T P pi_v for every u in U, v in V,
    no edge inside a side."""
    import scipy.sparse as sp
    alpha = np.full(k, alpha0 / k)
    pi_u = rng(seed, S_PI, 1).dirichlet(alpha, size=n_u)
    pi_v = rng(seed, S_PI, 2).dirichlet(alpha, size=n_v)
    P = np.full((k, k), q) + (p - q) * np.eye(k)
    eseed = int(rng(seed, S_EDGES, 2).integers(0, 2**63 - 1))
    src, dst, w = _pairs_general(pi_u, pi_v, False, poisson, p, q, eseed, pi_floor)
    m = sp.csr_matrix((w if poisson else np.ones_like(w), (src, dst)), shape=(n_u, n_v))
    C = CSR.from_scipy(m, implicit_ones=not poisson)
    return BipartiteInstance(k=k, alpha=alpha, P=P, pi_u=pi_u, pi_v=pi_v, C=C, CT=C.transpose(),
                             meta=dict(alpha0=alpha0, p=p, q=q, seed=seed, poisson=poisson))


# --------------------------------------------------------------------------
# LDA
# --------------------------------------------------------------------------
@dataclass
class LDAInstance:
    d: int
    k: int
    alpha: np.ndarray          # (k,)
    mu: np.ndarray             # (d, k) topic-word matrix, columns on the simplex
    h: np.ndarray              # (n, k) document mixtures
    lengths: np.ndarray        # (n,) document lengths
    C: CSR                     # (n, d) full word counts
    CT: CSR                    # (d, n)
    views: list                # three (n, d) count matrices, token positions mod 3
    meta: dict = field(default_factory=dict)


def lda(d: int, k: int, alpha0: float, beta: float, n_docs: int, mean_len: float,
        seed: int = BASE_SEED, mu: np.ndarray | None = None) -> LDAInstance:
    import scipy.sparse as sp
    alpha = np.full(k, alpha0 / k)
    if mu is None:
        mu = rng(seed, S_TOPICS).dirichlet(np.full(d, beta), size=k).T.copy()   # (d, k)
    h = rng(seed, S_MIX).dirichlet(alpha, size=n_docs)
    g = rng(seed, S_LENGTHS)
    lengths = g.poisson(mean_len, size=n_docs)
    bad = lengths < 3
    while bad.any():
        lengths[bad] = g.poisson(mean_len, size=int(bad.sum()))
        bad = lengths < 3
    n_tok = int(lengths.sum())
    doc = np.repeat(np.arange(n_docs, dtype=np.int64), lengths)
    start = np.zeros(n_docs + 1, dtype=np.int64)
    start[1:] = np.cumsum(lengths)
    pos = np.arange(n_tok, dtype=np.int64) - start[doc]
    view = (pos % 3).astype(np.int8)
    # topic of every token: inverse CDF on its document's mixture
    gt = rng(seed, S_TOKENS)
    topic = np.empty(n_tok, dtype=np.int32)
    cum = np.cumsum(h, axis=1)
    cum[:, -1] = 1.0
    chunk = 1 << 20
    for s in range(0, n_tok, chunk):
        e = min(n_tok, s + chunk)
        u = gt.random(e - s)
        topic[s:e] = np.minimum((u[:, None] >= cum[doc[s:e]]).sum(1), k - 1)
    # word of every token: inverse CDF on its topic's word distribution
    gw = rng(seed, S_WORDS)
    word = np.empty(n_tok, dtype=np.int32)
    u = gw.random(n_tok)
    for j in range(k):
        sel = np.nonzero(topic == j)[0]
        if len(sel) == 0:
            continue
        cdf = np.cumsum(mu[:, j])
        cdf[-1] = 1.0
        word[sel] = np.minimum(np.searchsorted(cdf, u[sel], side="right"), d - 1)
    ones = np.ones(n_tok, dtype=np.float32)
    full = sp.csr_matrix((ones, (doc, word)), shape=(n_docs, d))
    views = []
    for v in range(3):
        sel = view == v
        views.append(CSR.from_scipy(sp.csr_matrix((ones[sel], (doc[sel], word[sel])), shape=(n_docs, d))))
    C = CSR.from_scipy(full)
    return LDAInstance(d=d, k=k, alpha=alpha, mu=mu, h=h, lengths=lengths, C=C, CT=C.transpose(),
                       views=views, meta=dict(alpha0=alpha0, beta=beta, seed=seed))


# --------------------------------------------------------------------------
# Random quantities the method draws (passed to both sides as data)
# --------------------------------------------------------------------------
def projection(d: int, k_tilde: int, seed: int = BASE_SEED) -> np.ndarray:
    """Dense Gaussian projection S (d x k_tilde), FP64, row-major."""
    return rng(seed, S_PROJ).standard_normal((d, k_tilde))


def column_selection(d: int, k_tilde: int, seed: int = BASE_SEED):
    """Column-selection projection with random signs (for a sparse M2,
    Section 4.2): k_tilde distinct rows r_j of [d] and signs s_j in {-1, +1};
    S[r_j, j] = s_j and every other entry 0.  Returns (rows int32, signs FP64)."""
    g = rng(seed, S_PROJ, 7)
    rows = g.choice(d, size=k_tilde, replace=False).astype(np.int32)
    signs = np.where(g.random(k_tilde) < 0.5, -1.0, 1.0)
    return rows, signs


def selection_dense(rows: np.ndarray, signs: np.ndarray, d: int) -> np.ndarray:
    """The d x k_tilde matrix of a column selection."""
    S = np.zeros((d, len(rows)))
    S[rows, np.arange(len(rows))] = signs
    return S


def initial_factors(k: int, seed: int = BASE_SEED, restart: int = 0) -> np.ndarray:
    """Random k x k matrix with orthonormal columns (Haar): QR of a Gaussian,
    columns sign-fixed by the diagonal of R.  Column i is phi_i."""
    z = rng(seed, S_PHI0, restart).standard_normal((k, k))
    qm, r = np.linalg.qr(z)
    return qm * np.sign(np.diag(r))[None, :]


def permutations(n: int, passes: int, seed: int = BASE_SEED, sub: int = 0) -> np.ndarray:
    """passes x n int32: an independent uniform permutation of range(n) per pass."""
    g = rng(seed, S_PERM, sub)
    return np.stack([g.permutation(n) for _ in range(passes)]).astype(np.int32)


def dirichlet_alpha(k: int, alpha0: float) -> np.ndarray:
    return np.full(k, alpha0 / k)


# --------------------------------------------------------------------------
# Batched workload: many problems of whitened rows from a planted mixture
# --------------------------------------------------------------------------
def batched_table(n_problems: int = 256, ks=(16, 32, 64, 100, 128), n_lo: float = 1e3, n_hi: float = 1e5,
                  seed: int = BASE_SEED) -> list[dict]:
    """Shapes of the batched workload: k uniform over ks, n log-uniform in
    [n_lo, n_hi], half document-like problems (three views, alpha0 = 1) and half
    graph-like (one view, alpha0 = 0.1 up to n = 1e4, else 0.5), in random order."""
    g = rng(seed, S_MISC, 1)
    k = g.choice(np.asarray(ks), size=n_problems)
    n = np.exp(g.uniform(np.log(n_lo), np.log(n_hi), size=n_problems)).astype(np.int64)
    kinds = np.array(["lda"] * (n_problems // 2) + ["mmsb"] * (n_problems - n_problems // 2))
    g.shuffle(kinds)
    out = []
    for i in range(n_problems):
        a0 = 1.0 if kinds[i] == "lda" else (0.1 if n[i] <= 10_000 else 0.5)
        out.append(dict(kind=str(kinds[i]), n=int(n[i]), k=int(k[i]), alpha0=a0, views=3 if kinds[i] == "lda" else 1))
    return out


def planted_views(n: int, k: int, alpha0: float, views: int, seed: int = BASE_SEED, sub: int = 0,
                  device="cpu", noise: float = 0.3, ldy: int | None = None):
    """Whitened rows of a planted mixture, generated with torch on `device`:
    h_t ~ Dir(alpha0/k 1), M = sqrt(k) U with U a Haar orthonormal k x k matrix
    (the whitened topic directions when every alpha_i is alpha0/k), and for each
    view independently y_t = M h_t + (noise / sqrt(k)) N(0, I).  Returns the
    views as float32 tensors n x ldy (zero columns beyond k; one tensor three
    times when views == 1) and U.  Seeded: the torch generators are forked."""
    import torch
    ldy = ldy or k
    dev = torch.device(device)
    U = torch.as_tensor(initial_factors(k, seed, restart=10_000 + sub), dtype=torch.float32)
    M = (np.sqrt(k) * U).to(dev)
    devices = [dev] if dev.type == "cuda" else []
    with torch.random.fork_rng(devices=devices):
        torch.manual_seed(int(rng(seed, S_MISC, 2 + sub).integers(1 << 62)))
        conc = torch.full((k,), alpha0 / k, device=dev)
        h = torch.distributions.Dirichlet(conc).sample((n,))
        h = torch.nan_to_num(h, nan=1.0 / k)           # all-zero gamma draws at tiny alpha
        mean = h @ M.T
        out = []
        for _ in range(views):
            y = torch.zeros((n, ldy), dtype=torch.float32, device=dev)
            y[:, :k] = mean + (noise / np.sqrt(k)) * torch.randn((n, k), device=dev)
            out.append(y)
    if views == 1:
        out = out * 3
    return out[0], out[1], out[2], U


# --------------------------------------------------------------------------
# Configurations of the paper-shaped workloads
# --------------------------------------------------------------------------
CONFIGS = {
    # MMSB, n=1000, k=10, alpha0=0.1, p=0.3, q=0.05, X/A = 500/500, batch 100, 50 passes
    "mmsb_small": dict(kind="mmsb", n=1000, k=10, alpha0=0.1, p=0.3, q=0.05, n_x=500,
                       batch=100, passes=50),
    # LDA, d=10000, k=50, alpha0=1, beta=0.05, 100000 docs of length Poisson(200)
    "lda_medium": dict(kind="lda", d=10000, k=50, alpha0=1.0, beta=0.05, n_docs=100000,
                       mean_len=200.0, batch=100, passes=50),
    # MMSB, n=100000, k=100, alpha0=0.5, p=0.05, q=0.001, X/A = 50000/50000
    "mmsb_large": dict(kind="mmsb", n=100000, k=100, alpha0=0.5, p=0.05, q=0.001, n_x=50000,
                       batch=100, passes=50),
}


def make(name: str, seed: int = BASE_SEED, **over):
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    if cfg["kind"] == "mmsb":
        return mmsb(cfg["n"], cfg["k"], cfg["alpha0"], cfg["p"], cfg["q"], cfg["n_x"], seed=seed)
    return lda(cfg["d"], cfg["k"], cfg["alpha0"], cfg["beta"], cfg["n_docs"], cfg["mean_len"], seed=seed)
