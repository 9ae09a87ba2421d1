"""Seeded generators for the synthetic workloads of the FBPQ search.

Stand-in for SIFT-like data (the BIGANN base set, Section 4): 128-d points from
a 256-component Gaussian mixture with means uniform in [0, 128], standard
deviation 20, clipped to [0, 255] and rounded to integers (so every point is a
uint8 vector, like a SIFT descriptor).

Index construction follows the Multi-D-ADC recipe (Section 2.3): K-means on the
two halves gives the half codebooks C1 and C2 (equations q1, q2), the cell of a
point is the pair of nearest half centroids (equation Wij), the displacement
from the cell centroid (equation displacement) is PQ-encoded with M global
codebooks of Kc=256 words learnt by K-means on the training displacements, and
points are stored contiguously per cell with a start offset per cell. These
steps run offline; both the oracle and the GPU library consume their output.

Random draws use torch generators on the device the caller names (CPU in the
CPU tests, the GPU when a benchmark builds a large index); a seed fixes the
draws for a given device type. Seeds: 0 mixture means and training sample,
1 base points, 2 queries, 3 per-query L and k, 4 Zipf occupancy and codes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

KC = 256


@dataclass
class Index:
    """A multi-index with PQ-encoded displacements, in host memory.

    C1, C2:  float32 [T, D/2]       half codebooks
    R:       float32 [M, Kc, D/M]   displacement codebooks R_1..R_M
    offsets: int64   [T*T + 1]      start of cell c = i*T + j in storage order
    codes:   uint8   [N, M]         PQ code of each stored point
    ids:     uint32  [N]            original point id of each stored point
    base:    optional [N, D] raw vectors indexed by original id (uint8 or
             float32), kept for exact-NN recall
    QL, SL:  optional float32 [T, M/2, Kc, D/M] local codebooks (HBPQ): QL[i]
             codes the first half of the displacements in the cells of row i,
             SL[j] the second half in the cells of column j; R is then unused
    Rot:     optional float32 [D, D] orthogonal rotation (OPQ): the index lives
             in the rotated space and a query q enters it as Rot q
    """

    D: int
    T: int
    M: int
    C1: np.ndarray
    C2: np.ndarray
    R: np.ndarray
    offsets: np.ndarray
    codes: np.ndarray
    ids: np.ndarray
    Kc: int = KC
    base: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)
    QL: Optional[np.ndarray] = None
    SL: Optional[np.ndarray] = None
    Rot: Optional[np.ndarray] = None

    @property
    def local(self) -> bool:
        return self.QL is not None

    @property
    def N(self) -> int:
        return int(self.codes.shape[0])

    def check(self) -> None:
        D, T, M, Kc = self.D, self.T, self.M, self.Kc
        assert D % 2 == 0 and M % 2 == 0 and D % M == 0
        assert self.C1.shape == (T, D // 2) and self.C1.dtype == np.float32
        assert self.C2.shape == (T, D // 2) and self.C2.dtype == np.float32
        assert self.R.shape == (M, Kc, D // M) and self.R.dtype == np.float32
        assert self.offsets.shape == (T * T + 1,) and self.offsets.dtype == np.int64
        assert self.codes.ndim == 2 and self.codes.shape[1] == M and self.codes.dtype == np.uint8
        assert self.ids.shape == (self.N,) and self.ids.dtype == np.uint32
        assert self.offsets[0] == 0 and self.offsets[-1] == self.N
        assert np.all(np.diff(self.offsets) >= 0)
        if self.QL is not None or self.SL is not None:
            shp = (T, M // 2, Kc, D // M)
            assert self.QL is not None and self.SL is not None
            assert self.QL.shape == shp and self.QL.dtype == np.float32
            assert self.SL.shape == shp and self.SL.dtype == np.float32
        if self.Rot is not None:
            assert self.Rot.shape == (D, D) and self.Rot.dtype == np.float32


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    return g


def gmm_means(seed: int = 0, ncomp: int = 256, D: int = 128) -> torch.Tensor:
    """Mixture means, uniform in [0, 128]^D (drawn on the CPU, float32)."""
    g = _gen(seed, "cpu")
    return torch.rand(ncomp, D, generator=g, dtype=torch.float32) * 128.0


def sample_points(n: int, means: torch.Tensor, seed: int, device="cpu",
                  sigma: float = 20.0, chunk: int = 1 << 21) -> torch.Tensor:
    """n points of the mixture as uint8 [n, D] on `device` (equal weights)."""
    device = torch.device(device)
    g = _gen(seed, device)
    mu = means.to(device)
    ncomp, D = mu.shape
    out = torch.empty(n, D, dtype=torch.uint8, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        comp = torch.randint(0, ncomp, (e - s,), generator=g, device=device)
        x = torch.randn(e - s, D, generator=g, device=device, dtype=torch.float32)
        x.mul_(sigma).add_(mu[comp])
        out[s:e] = x.clamp_(0.0, 255.0).round_().to(torch.uint8)
    return out


def _nearest(X: torch.Tensor, Cb: torch.Tensor, chunk: int) -> torch.Tensor:
    """Index of the nearest row of Cb for each row of X (first index on ties)."""
    cn = (Cb * Cb).sum(1)
    out = torch.empty(X.shape[0], dtype=torch.int64, device=X.device)
    for s in range(0, X.shape[0], chunk):
        x = X[s:s + chunk]
        d = cn[None, :] - 2.0 * (x @ Cb.T)
        out[s:s + chunk] = d.argmin(1)
    return out


def _lloyd(X: torch.Tensor, K: int, iters: int, g: torch.Generator, chunk: int) -> torch.Tensor:
    """Lloyd K-means: init = first K rows of a seeded permutation of X; an empty
    cluster keeps its previous centroid."""
    n = X.shape[0]
    perm = torch.randperm(n, generator=g, device=g.device)
    C = X[perm[:K].to(X.device)].clone()
    for _ in range(iters):
        a = _nearest(X, C, chunk)
        s = torch.zeros_like(C).index_add_(0, a, X)
        cnt = torch.bincount(a, minlength=K).to(X.dtype)
        nz = cnt > 0
        C[nz] = s[nz] / cnt[nz, None]
    return C


def _csr(cell: torch.Tensor, ncell: int):
    order = torch.sort(cell, stable=True).indices
    counts = torch.bincount(cell, minlength=ncell)
    offsets = torch.zeros(ncell + 1, dtype=torch.int64, device=cell.device)
    offsets[1:] = torch.cumsum(counts, 0)
    return order, offsets


def build_index(base: torch.Tensor, T: int, M: int, seed: int = 0, train_n: int = 20000,
                iters: int = 10, keep_base: bool = True, chunk: Optional[int] = None) -> Index:
    """Train C1, C2 and R on a `train_n` sample of `base` and encode every point.

    base: uint8 [N, D] on any device; the computation runs on that device.
    """
    device = base.device
    N, D = base.shape
    assert D % 2 == 0 and M % 2 == 0 and D % M == 0
    h, ds = D // 2, D // M
    if chunk is None:
        chunk = max(1024, (1 << 27) // max(T, KC)) if device.type != "cpu" else 4096
    g = _gen(seed, device)
    ntr = min(train_n, N)
    sel = torch.randperm(N, generator=g, device=device)[:ntr]
    Xtr = base[sel].to(torch.float32)
    C1 = _lloyd(Xtr[:, :h].contiguous(), T, iters, g, chunk)
    C2 = _lloyd(Xtr[:, h:].contiguous(), T, iters, g, chunk)
    i_tr = _nearest(Xtr[:, :h].contiguous(), C1, chunk)
    j_tr = _nearest(Xtr[:, h:].contiguous(), C2, chunk)
    Dtr = Xtr - torch.cat([C1[i_tr], C2[j_tr]], 1)
    R = torch.stack([_lloyd(Dtr[:, k * ds:(k + 1) * ds].contiguous(), KC, iters, g, chunk)
                     for k in range(M)])
    codes = torch.empty(N, M, dtype=torch.uint8, device=device)
    cell = torch.empty(N, dtype=torch.int64, device=device)
    big = 1 << 20 if device.type != "cpu" else 1 << 16
    for s in range(0, N, big):
        x = base[s:s + big].to(torch.float32)
        i = _nearest(x[:, :h].contiguous(), C1, chunk)
        j = _nearest(x[:, h:].contiguous(), C2, chunk)
        d = x - torch.cat([C1[i], C2[j]], 1)
        for k in range(M):
            codes[s:s + big, k] = _nearest(d[:, k * ds:(k + 1) * ds].contiguous(), R[k], chunk).to(torch.uint8)
        cell[s:s + big] = i * T + j
    order, offsets = _csr(cell, T * T)
    ix = Index(D=D, T=T, M=M,
               C1=C1.cpu().numpy(), C2=C2.cpu().numpy(), R=R.cpu().numpy(),
               offsets=offsets.cpu().numpy(),
               codes=codes[order].cpu().numpy(),
               ids=order.to(torch.int32).cpu().numpy().view(np.uint32) if N < 2**31
               else order.cpu().numpy().astype(np.uint32),
               base=base.cpu().numpy() if keep_base else None,
               meta=dict(kind="gmm", seed=seed, train_n=ntr, iters=iters))
    ix.check()
    return ix


def random_rotation(D: int, seed: int = 23) -> np.ndarray:
    """A seeded orthogonal D x D matrix (float32): the Q factor of a Gaussian
    matrix, columns signed so that R's diagonal is positive (a unique choice)."""
    g = _gen(seed, "cpu")
    a = torch.randn(D, D, generator=g, dtype=torch.float64)
    q, r = torch.linalg.qr(a)
    q = q * torch.sign(torch.diagonal(r))[None, :]
    return q.to(torch.float32).numpy()


def make_queries(nq: int, means: torch.Tensor, seed: int = 2, device="cpu") -> np.ndarray:
    """nq queries from the same mixture, float32 [nq, D] in host memory."""
    return sample_points(nq, means, seed, device).to(torch.float32).cpu().numpy()


def draw_L_k(nq: int, seed: int = 3, L_lo: int = 1000, L_hi: int = 100000,
             ks=(1, 10, 100)):
    """Per-query budgets: L log-uniform in [L_lo, L_hi], k uniform over `ks`."""
    g = _gen(seed, "cpu")
    u = torch.rand(nq, generator=g, dtype=torch.float64)
    L = torch.exp(math.log(L_lo) + u * (math.log(L_hi) - math.log(L_lo))).round().to(torch.int64)
    kk = torch.tensor(ks, dtype=torch.int32)[torch.randint(0, len(ks), (nq,), generator=g)]
    return L.numpy(), kk.numpy()


def _from_cells(D, T, M, C1, C2, R, cell, codes, base, meta) -> Index:
    cell_t = torch.as_tensor(cell, dtype=torch.int64)
    order, offsets = _csr(cell_t, T * T)
    o = order.numpy()
    ix = Index(D=D, T=T, M=M, C1=C1, C2=C2, R=R, offsets=offsets.numpy(),
               codes=np.ascontiguousarray(codes[o]), ids=o.astype(np.uint32),
               base=base, meta=meta)
    ix.check()
    return ix


def lossless_index(N: int, T: int, M: int, D: int = 16, seed: int = 7, dup: int = 0,
                   shuffle_ids: bool = False) -> Index:
    """Points built exactly as [c1_i; c2_j] + [R_1(b_1); ...; R_M(b_M)].

    Every coordinate is a small integer, so the reconstruction of equation
    (approximation) is exact and the raw vectors (`base`, float32) equal it.
    The last `dup` points repeat earlier points exactly (equal distances);
    `shuffle_ids` relabels the points with a random permutation so that ids
    are not ascending in storage order.
    """
    g = _gen(seed, "cpu")
    h, ds = D // 2, D // M
    C1 = torch.randint(-40, 41, (T, h), generator=g).to(torch.float32).numpy()
    C2 = torch.randint(-40, 41, (T, h), generator=g).to(torch.float32).numpy()
    R = torch.randint(-8, 9, (M, KC, ds), generator=g).to(torch.float32).numpy()
    i = torch.randint(0, T, (N,), generator=g).numpy()
    j = torch.randint(0, T, (N,), generator=g).numpy()
    codes = torch.randint(0, KC, (N, M), generator=g).to(torch.uint8).numpy()
    if dup:
        src = torch.randint(0, N - dup, (dup,), generator=g).numpy()
        i[N - dup:], j[N - dup:], codes[N - dup:] = i[src], j[src], codes[src]
    base = np.concatenate([C1[i], C2[j]], 1)
    for k in range(M):
        base[:, k * ds:(k + 1) * ds] += R[k][codes[:, k]]
    ix = _from_cells(D, T, M, C1, C2, R, i * T + j, codes, base.astype(np.float32),
                     dict(kind="lossless", seed=seed))
    if shuffle_ids:
        perm = torch.randperm(N, generator=g).numpy()
        newbase = np.empty_like(ix.base)
        newbase[perm] = ix.base
        ix.ids = perm[ix.ids.astype(np.int64)].astype(np.uint32)
        ix.base = newbase
    return ix


def lossless_local_index(N: int, T: int, M: int, D: int = 16, seed: int = 13, dup: int = 0) -> Index:
    """Points built exactly as [c1_i + (Q^i_1(b_1), ..., Q^i_{M/2}(b_{M/2}));
    c2_j + (S^j_1(b_{M/2+1}), ...)] with local codebooks that differ from
    centroid to centroid (equation residual of Section 3.2). Every coordinate is
    a small integer, so the reconstruction is exact and `base` equals it."""
    g = _gen(seed, "cpu")
    h, ds, mh = D // 2, D // M, M // 2
    C1 = torch.randint(-40, 41, (T, h), generator=g).to(torch.float32).numpy()
    C2 = torch.randint(-40, 41, (T, h), generator=g).to(torch.float32).numpy()
    R = np.zeros((M, KC, ds), np.float32)  # unused with local codebooks
    QL = torch.randint(-8, 9, (T, mh, KC, ds), generator=g).to(torch.float32).numpy()
    SL = torch.randint(-8, 9, (T, mh, KC, ds), generator=g).to(torch.float32).numpy()
    i = torch.randint(0, T, (N,), generator=g).numpy()
    j = torch.randint(0, T, (N,), generator=g).numpy()
    codes = torch.randint(0, KC, (N, M), generator=g).to(torch.uint8).numpy()
    if dup:
        src = torch.randint(0, N - dup, (dup,), generator=g).numpy()
        i[N - dup:], j[N - dup:], codes[N - dup:] = i[src], j[src], codes[src]
    base = np.concatenate([C1[i], C2[j]], 1)
    for k in range(mh):
        base[:, k * ds:(k + 1) * ds] += QL[i, k, codes[:, k]]
        base[:, h + k * ds:h + (k + 1) * ds] += SL[j, k, codes[:, mh + k]]
    ix = _from_cells(D, T, M, C1, C2, R, i * T + j, codes, base.astype(np.float32),
                     dict(kind="lossless_local", seed=seed))
    ix.QL, ix.SL = QL, SL
    ix.check()
    return ix


def with_local_codebooks(ix: Index, seed: int = 17, scale: float = 0.25) -> Index:
    """The same index with local codebooks: Q^i_k = R_k + noise and S^j_k =
    R_{M/2+k} + noise, seeded, the noise `scale` times the codebook's standard
    deviation. The codes stay the global encoding (the per-cell training of
    Section 3.2 is outside this generator); the search cost does not depend on
    how the codes were chosen."""
    g = _gen(seed, "cpu")
    T, M, D = ix.T, ix.M, ix.D
    mh, ds = M // 2, D // M
    R = torch.from_numpy(ix.R)
    sd = float(R.std()) * scale
    QL = (R[:mh][None] + sd * torch.randn((T, mh, KC, ds), generator=g)).to(torch.float32).numpy()
    SL = (R[mh:][None] + sd * torch.randn((T, mh, KC, ds), generator=g)).to(torch.float32).numpy()
    out = Index(D=D, T=T, M=M, C1=ix.C1, C2=ix.C2, R=ix.R, offsets=ix.offsets, codes=ix.codes,
                ids=ix.ids, Kc=ix.Kc, base=ix.base, meta=dict(ix.meta, local_seed=seed), QL=QL, SL=SL)
    out.check()
    return out


def random_index(N: int, T: int, M: int, D: int = 16, seed: int = 11,
                 empty_frac: float = 0.0, int_valued: bool = False) -> Index:
    """Random centroids, codebooks, cells and codes (no training), for structure
    tests. A fraction `empty_frac` of the cells is kept empty."""
    g = _gen(seed, "cpu")
    h, ds = D // 2, D // M
    if int_valued:
        C1 = torch.randint(0, 32, (T, h), generator=g).to(torch.float32).numpy()
        C2 = torch.randint(0, 32, (T, h), generator=g).to(torch.float32).numpy()
        R = torch.randint(-4, 5, (M, KC, ds), generator=g).to(torch.float32).numpy()
    else:
        C1 = (torch.rand(T, h, generator=g) * 100).numpy()
        C2 = (torch.rand(T, h, generator=g) * 100).numpy()
        R = (torch.randn(M, KC, ds, generator=g) * 10).numpy().astype(np.float32)
    allowed = torch.randperm(T * T, generator=g)[:max(1, int(round(T * T * (1 - empty_frac))))]
    cell = allowed[torch.randint(0, allowed.numel(), (N,), generator=g)].numpy()
    codes = torch.randint(0, KC, (N, M), generator=g).to(torch.uint8).numpy()
    return _from_cells(D, T, M, C1.astype(np.float32), C2.astype(np.float32), R, cell, codes, None,
                       dict(kind="random", seed=seed))


def tiny_index(T: int, counts: np.ndarray, M: int = 2, D: int = 4, seed: int = 5,
               C1: Optional[np.ndarray] = None, C2: Optional[np.ndarray] = None) -> Index:
    """Index with a prescribed number of points per cell (counts[T*T]) and
    optional prescribed centroids, for traversal edge cases and forced ties."""
    g = _gen(seed, "cpu")
    h, ds = D // 2, D // M
    if C1 is None:
        C1 = torch.randint(0, 6, (T, h), generator=g).to(torch.float32).numpy()
    if C2 is None:
        C2 = torch.randint(0, 6, (T, h), generator=g).to(torch.float32).numpy()
    R = torch.randint(-3, 4, (M, KC, ds), generator=g).to(torch.float32).numpy()
    counts = np.asarray(counts, dtype=np.int64).reshape(T * T)
    cell = np.repeat(np.arange(T * T, dtype=np.int64), counts)
    perm = torch.randperm(cell.size, generator=g).numpy()
    cell = cell[perm]
    codes = torch.randint(0, KC, (cell.size, M), generator=g).to(torch.uint8).numpy()
    return _from_cells(D, T, M, np.asarray(C1, np.float32), np.asarray(C2, np.float32), R,
                       cell, codes, None, dict(kind="tiny", seed=seed))


def zipf_index(N: int, T: int, M: int, D: int = 128, s: float = 1.1, seed: int = 4,
               codebook_seed: int = 0, device="cpu") -> Index:
    """Served-scale synthetic index: the cell of each point is a Zipf(s) rank over
    the T*T cells mapped to a cell id by a seeded permutation; codes are uniform
    bytes; ids are storage positions. Centroids and codebooks are trained as in
    `build_index` on a 20k mixture sample with the given T."""
    device = torch.device(device)
    means = gmm_means(0, 256, D)
    tr = sample_points(20000, means, 1, device)
    ref = build_index(tr, T, M, seed=codebook_seed, train_n=20000, keep_base=False)
    g = _gen(seed, device)
    C = T * T
    # inverse-CDF draw of Zipf ranks (FP64 CDF over all C ranks)
    cdf = torch.arange(1, C + 1, device=device, dtype=torch.float64).pow_(-s).cumsum_(0)
    cdf /= cdf[-1].clone()
    counts = torch.zeros(C, dtype=torch.int64, device=device)
    step = 1 << 26
    for s0 in range(0, N, step):
        n = min(step, N - s0)
        u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
        r = torch.searchsorted(cdf, u).clamp_(max=C - 1)
        counts += torch.bincount(r, minlength=C)
        del u, r
    del cdf
    perm = torch.randperm(C, generator=g, device=device)
    cell_counts = torch.empty_like(counts)
    cell_counts[perm] = counts
    offsets = torch.zeros(C + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(cell_counts, 0)
    codes = torch.randint(0, 256, (N, M), generator=g, device=device, dtype=torch.uint8)
    ix = Index(D=D, T=T, M=M, C1=ref.C1, C2=ref.C2, R=ref.R,
               offsets=offsets.cpu().numpy(), codes=codes.cpu().numpy(),
               ids=np.arange(N, dtype=np.uint32), base=None,
               meta=dict(kind="zipf", s=s, seed=seed))
    return ix
