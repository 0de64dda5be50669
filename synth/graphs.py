"""Seeded synthetic graph and label generators.

These produce the *inputs* of the segmentation method (a weighted undirected graph in
CSR form, the labelled node set, its labels and a ground-truth class per node).  They
hold none of the method's arithmetic: no Laplacian, objective, gradient, oracle or
step size appears here.  Both the oracle and the GPU path consume what they return.

All randomness comes from numpy's PCG64 seeded explicitly; the same seed gives the
same graph on every machine (the k-NN builder is the one exception: its neighbour
search runs in float32 and may resolve exact distance ties differently on different
BLAS back ends, which is harmless because each test passes one and the same instance
to both implementations).

The weight formula used for image-like grids is the Gaussian similarity of Section 1
of the paper, w_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)), applied to pixel intensities.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    """Undirected weighted graph in CSR form (symmetric pattern and values).

    indptr  int64[n+1], indices int32[nnz] (sorted within each row, no duplicates),
    data    float64[nnz] (w_ij > 0), truth int32[n] (ground-truth class, or -1),
    K       number of classes.
    """

    n: int
    K: int
    indptr: np.ndarray
    indices: np.ndarray
    data: np.ndarray
    truth: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])


def rng_for(seed: int, stream: int) -> np.random.Generator:
    """Independent sub-stream `stream` of master seed `seed` (PCG64)."""
    ss = np.random.SeedSequence([int(seed), int(stream)])
    return np.random.Generator(np.random.PCG64(ss))


def _csr_from_edges(n: int, a: np.ndarray, b: np.ndarray, w: np.ndarray) -> tuple:
    """Symmetric CSR from an undirected edge list (a_e != b_e, no duplicate pairs)."""
    rows = np.concatenate([a, b]).astype(np.int64)
    cols = np.concatenate([b, a]).astype(np.int64)
    vals = np.concatenate([w, w]).astype(np.float64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    vals = vals[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    indptr[1:] = np.cumsum(np.bincount(rows, minlength=n))
    return indptr, cols, vals


def _dedup_pairs(n: int, a: np.ndarray, b: np.ndarray) -> tuple:
    """Drop self-pairs, order each pair (min, max) and remove duplicates."""
    keep = a != b
    a, b = a[keep], b[keep]
    lo = np.minimum(a, b).astype(np.int64)
    hi = np.maximum(a, b).astype(np.int64)
    key = np.unique(lo * n + hi)
    return (key // n), (key % n)


def sbm(sizes, p_in: float, p_out: float, seed: int, permute: bool = True, K: int | None = None) -> Graph:
    """Stochastic block model with unit weights and no self-loops.

    Edge counts per block pair are binomial, endpoints uniform, duplicates dropped
    (O(nnz) sampling; for small graphs each pair is an independent Bernoulli draw).
    Node order is randomly permuted so that communities are not contiguous.
    """
    sizes = [int(s) for s in sizes]
    n = int(sum(sizes))
    Kc = len(sizes) if K is None else K
    rg = rng_for(seed, 1)
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    truth = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    A, B = [], []
    if n <= 4000:
        iu, ju = np.triu_indices(n, k=1)
        same = truth[iu] == truth[ju]
        p = np.where(same, p_in, p_out)
        hit = rg.random(iu.shape[0]) < p
        A.append(iu[hit].astype(np.int64))
        B.append(ju[hit].astype(np.int64))
    else:
        for x in range(len(sizes)):
            for y in range(x, len(sizes)):
                if x == y:
                    pairs = sizes[x] * (sizes[x] - 1) // 2
                    m = rg.binomial(pairs, p_in)
                    a = rg.integers(0, sizes[x], size=int(m * 1.001) + 16) + starts[x]
                    b = rg.integers(0, sizes[x], size=a.shape[0]) + starts[x]
                else:
                    pairs = sizes[x] * sizes[y]
                    m = rg.binomial(pairs, p_out)
                    a = rg.integers(0, sizes[x], size=int(m * 1.001) + 16) + starts[x]
                    b = rg.integers(0, sizes[y], size=a.shape[0]) + starts[y]
                lo, hi = _dedup_pairs(n, a, b)
                if lo.shape[0] > m:
                    sel = rg.choice(lo.shape[0], size=m, replace=False)
                    sel.sort()
                    lo, hi = lo[sel], hi[sel]
                A.append(lo)
                B.append(hi)
    a = np.concatenate(A)
    b = np.concatenate(B)
    if permute:
        perm = rng_for(seed, 2).permutation(n).astype(np.int64)
        a, b = perm[a], perm[b]
        t2 = np.empty_like(truth)
        t2[perm] = truth
        truth = t2
    indptr, indices, data = _csr_from_edges(n, a, b, np.ones(a.shape[0]))
    return Graph(n=n, K=Kc, indptr=indptr, indices=indices, data=data, truth=truth,
                 name=f"sbm(n={n},K={len(sizes)})")


def sbm_by_degree(n: int, K: int, avg_degree: float, ratio: float, seed: int) -> Graph:
    """SBM with K near-equal blocks, expected degree `avg_degree` and p_in/p_out = `ratio`."""
    sizes = [n // K + (1 if c < n % K else 0) for c in range(K)]
    m = n / K
    # expected degree = p_in (m - 1) + p_out (n - m), p_in = ratio * p_out
    p_out = avg_degree / (ratio * (m - 1) + (n - m))
    p_in = ratio * p_out
    return sbm(sizes, min(p_in, 1.0), min(p_out, 1.0), seed)


def lfr_like(n: int, K: int, avg_degree: float, mu: float, seed: int, tau1: float = 2.5, tau2: float = 1.5,
             max_degree: int = 50) -> Graph:
    """A graph with the shape of an LFR benchmark network: power-law degrees (exponent tau1,
    mean about `avg_degree`, at most `max_degree`), K communities of power-law sizes (exponent
    tau2, at least 3 nodes), and a fraction `mu` of each node's edge ends placed outside its
    community.  Edge ends are paired at random (inside the community, or over all outside
    ends), self-pairs and duplicates are dropped, weights are 1, nodes are randomly ordered."""
    rg = rng_for(seed, 11)
    if K * 3 > n:
        raise ValueError("need at least 3 nodes per community")
    # community sizes: power law truncated to [n/(4K), 8n/K], rescaled to sum to n
    lo, hi = max(3.0, n / (4.0 * K)), min(float(n), 8.0 * n / K)
    e = 1.0 - tau2
    x = rg.random(K)
    raw = (lo ** e + x * (hi ** e - lo ** e)) ** (1.0 / e)
    sizes = np.maximum(3, np.floor(raw / raw.sum() * n).astype(np.int64))
    while sizes.sum() > n:
        sizes[np.argmax(sizes)] -= 1
    sizes[np.argmin(sizes)] += n - sizes.sum()
    truth = np.repeat(np.arange(K, dtype=np.int32), sizes)
    # degrees: power law, clipped to [1, max_degree]; the scale is set so that the clipped
    # mean is avg_degree
    y = (1.0 - rg.random(n)) ** (-1.0 / (tau1 - 1.0))
    xmin = avg_degree * (tau1 - 2.0) / (tau1 - 1.0)
    for _ in range(4):
        d = np.clip(np.floor(xmin * y + 0.5), 1, max_degree)
        xmin *= avg_degree / d.mean()
    deg = np.clip(np.floor(xmin * y + 0.5), 1, max_degree).astype(np.int64)
    n_out = rg.binomial(deg, mu)
    n_in = deg - n_out
    A, B = [], []
    starts = np.concatenate([[0], np.cumsum(sizes)])
    for c in range(K):
        nodes = np.arange(starts[c], starts[c + 1])
        ends = np.repeat(nodes, n_in[nodes])
        rg.shuffle(ends)
        m = ends.shape[0] // 2
        A.append(ends[:m])
        B.append(ends[m:2 * m])
    ends = np.repeat(np.arange(n), n_out)
    rg.shuffle(ends)
    m = ends.shape[0] // 2
    A.append(ends[:m])
    B.append(ends[m:2 * m])
    a, b = _dedup_pairs(n, np.concatenate(A), np.concatenate(B))
    perm = rng_for(seed, 12).permutation(n).astype(np.int64)
    a, b = perm[a], perm[b]
    t2 = np.empty_like(truth)
    t2[perm] = truth
    indptr, indices, data = _csr_from_edges(n, a, b, np.ones(a.shape[0]))
    return Graph(n=n, K=K, indptr=indptr, indices=indices, data=data, truth=t2,
                 name=f"lfr_like(n={n},K={K},mu={mu})")


def gaussian_mixture_knn(n: int, d: int, K: int, k: int, seed: int, center_scale: float = 2.0,
                         sigma: float = 1.0, device: str = "cpu") -> Graph:
    """k-NN graph of an isotropic Gaussian mixture.

    Centres mu_c ~ N(0, center_scale^2 I_d); n/K points per class x = mu_c + sigma N(0, I).
    Exact k nearest neighbours (self excluded) in float32 by blocked distance products,
    symmetrised by union.  w_ij = exp(-||x_i - x_j||^2 / (s_i s_j)) with s_i the distance
    from i to its k-th neighbour (a local-scaling reading of the Gaussian similarity).
    """
    import torch

    rg = rng_for(seed, 1)
    per = [n // K + (1 if c < n % K else 0) for c in range(K)]
    truth = np.repeat(np.arange(K, dtype=np.int32), per)
    mu = rg.standard_normal((K, d)) * center_scale
    X = (mu[truth] + sigma * rg.standard_normal((n, d))).astype(np.float32)
    perm = rng_for(seed, 2).permutation(n)
    X = X[perm]
    truth = truth[perm]
    Xt = torch.from_numpy(X).to(device)
    sq = (Xt * Xt).sum(1)
    nbr = np.empty((n, k), dtype=np.int64)
    dist = np.empty((n, k), dtype=np.float64)
    bs = 4096 if device != "cpu" else 2048
    for s0 in range(0, n, bs):
        s1 = min(n, s0 + bs)
        D = sq[s0:s1, None] + sq[None, :] - 2.0 * (Xt[s0:s1] @ Xt.T)
        D[torch.arange(s1 - s0), torch.arange(s0, s1)] = float("inf")
        vals, idx = torch.topk(D, k, dim=1, largest=False, sorted=True)
        nbr[s0:s1] = idx.cpu().numpy()
        dist[s0:s1] = np.sqrt(np.maximum(vals.double().cpu().numpy(), 0.0))
    # exact squared distances of the selected pairs in float64 (for the weights)
    a = np.repeat(np.arange(n, dtype=np.int64), k)
    b = nbr.reshape(-1)
    lo, hi = _dedup_pairs(n, a, b)
    X64 = X.astype(np.float64)
    d2 = np.empty(lo.shape[0])
    for s0 in range(0, lo.shape[0], 1 << 18):
        s1 = min(lo.shape[0], s0 + (1 << 18))
        diff = X64[lo[s0:s1]] - X64[hi[s0:s1]]
        d2[s0:s1] = np.einsum("ij,ij->i", diff, diff)
    s = dist[:, k - 1]
    w = np.exp(-d2 / (s[lo] * s[hi]))
    w = np.maximum(w, 1e-300)
    indptr, indices, data = _csr_from_edges(n, lo, hi, w)
    return Graph(n=n, K=K, indptr=indptr, indices=indices, data=data, truth=truth,
                 name=f"knn(n={n},d={d},K={K},k={k})")


def region_image(H: int, W: int, K: int, seed: int, noise: float = 0.05) -> tuple:
    """Synthetic K-region intensity image: Voronoi cells of K random seeds, levels evenly
    spaced in [0.1, 0.9] plus Gaussian noise.  Returns (image float64[H, W], truth int32[H*W])."""
    rg = rng_for(seed, 3)
    pts = rg.random((K, 2)) * np.array([H, W])
    yy, xx = np.mgrid[0:H, 0:W]
    d2 = (yy[..., None] - pts[:, 0]) ** 2 + (xx[..., None] - pts[:, 1]) ** 2
    region = np.argmin(d2, axis=2).astype(np.int32)
    levels = np.linspace(0.1, 0.9, K)
    img = levels[region] + noise * rg.standard_normal((H, W))
    return img, region.reshape(-1)


def color_image(H: int, W: int, K: int, seed: int, noise: float = 0.1, min_sep: float = 0.25) -> tuple:
    """Synthetic K-region colour image: Voronoi cells of K random seed points, each region one
    RGB colour drawn in [0.1, 0.9]^3 (redrawn until every pair is min_sep apart), plus
    Gaussian noise of standard deviation `noise` per channel.  Returns (features float64
    [H*W, 3], the RGB of each pixel in row-major order, truth int32[H*W])."""
    rg = rng_for(seed, 6)
    pts = rg.random((K, 2)) * np.array([H, W])
    yy, xx = np.mgrid[0:H, 0:W]
    d2 = (yy[..., None] - pts[:, 0]) ** 2 + (xx[..., None] - pts[:, 1]) ** 2
    region = np.argmin(d2, axis=2).astype(np.int32).reshape(-1)
    cols = np.zeros((K, 3))
    for c in range(K):
        for _ in range(1000):
            cand = 0.1 + 0.8 * rg.random(3)
            if c == 0 or np.min(np.linalg.norm(cols[:c] - cand, axis=1)) >= min_sep:
                break
        cols[c] = cand
    feats = cols[region] + noise * rg.standard_normal((H * W, 3))
    return feats, region


def grid_graph(H: int, W: int, img: np.ndarray, neighbours: int = 4, sigma_i: float = 0.1) -> tuple:
    """4- or 8-neighbour pixel grid with w = exp(-(I_p - I_q)^2 / (2 sigma_i^2))."""
    n = H * W
    idx = np.arange(n, dtype=np.int64).reshape(H, W)
    offs = [(0, 1), (1, 0)] if neighbours == 4 else [(0, 1), (1, 0), (1, 1), (1, -1)]
    A, B, Wt = [], [], []
    for dy, dx in offs:
        y0, y1 = 0, H - dy
        x0, x1 = max(0, -dx), W - max(0, dx)
        a = idx[y0:y1, x0:x1].reshape(-1)
        b = idx[y0 + dy:y1 + dy, x0 + dx:x1 + dx].reshape(-1)
        ia = img[y0:y1, x0:x1].reshape(-1)
        ib = img[y0 + dy:y1 + dy, x0 + dx:x1 + dx].reshape(-1)
        A.append(a)
        B.append(b)
        Wt.append(np.exp(-((ia - ib) ** 2) / (2.0 * sigma_i * sigma_i)))
    a = np.concatenate(A)
    b = np.concatenate(B)
    w = np.maximum(np.concatenate(Wt), 1e-300)
    return _csr_from_edges(n, a, b, w)


def image_grid(n_target: int, K: int, seed: int, neighbours: int = 4, side: int | None = None) -> Graph:
    """Grid graph over a synthetic K-region image with about n_target pixels."""
    if side is not None:
        H = W = int(side)
    else:
        H = max(2, int(math.isqrt(int(n_target))))
        W = max(2, -(-int(n_target) // H))
    img, truth = region_image(H, W, K, seed)
    indptr, indices, data = grid_graph(H, W, img, neighbours)
    g = Graph(n=H * W, K=K, indptr=indptr, indices=indices, data=data, truth=truth,
              name=f"grid{neighbours}({H}x{W},K={K})")
    g.shape = (H, W)  # type: ignore[attr-defined]
    return g


def path_graph(n: int, K: int) -> Graph:
    """Path 0 - 1 - ... - (n-1) with unit weights (used by worked examples)."""
    a = np.arange(n - 1, dtype=np.int64)
    indptr, indices, data = _csr_from_edges(n, a, a + 1, np.ones(n - 1))
    return Graph(n=n, K=K, indptr=indptr, indices=indices, data=data,
                 truth=np.full(n, -1, np.int32), name=f"path({n})")


def stratified_labels(truth: np.ndarray, K: int, frac: float, seed: int) -> tuple:
    """max(1, round(frac * |C_c|)) labelled nodes per class, sampled without replacement.
    Returns (labelled_idx int32 sorted, labels int32)."""
    rg = rng_for(seed, 4)
    idx, lab = [], []
    for c in range(K):
        members = np.flatnonzero(truth == c)
        if members.size == 0:
            continue
        m = max(1, int(round(frac * members.size)))
        pick = rg.choice(members, size=min(m, members.size), replace=False)
        idx.append(pick)
        lab.append(np.full(pick.shape[0], c, np.int32))
    idx = np.concatenate(idx).astype(np.int32)
    lab = np.concatenate(lab)
    order = np.argsort(idx)
    return idx[order], lab[order]


def scribble_labels(truth: np.ndarray, H: int, W: int, K: int, frac: float, seed: int,
                    stroke_len: int | None = None) -> tuple:
    """Random-walk strokes inside each region, about frac * n pixels split evenly over the
    classes present.  stroke_len=None draws one long stroke per class (restarted only at
    random when it runs into the region's border); an integer starts a new stroke at a random
    pixel of the class after every stroke_len steps.  Returns (labelled_idx int32 sorted,
    labels int32)."""
    rg = rng_for(seed, 5)
    region = truth.reshape(H, W)
    total = max(K, int(round(frac * H * W)))
    per = max(1, total // K)
    chosen = np.zeros(H * W, dtype=bool)
    steps = np.array([(0, 1), (1, 0), (0, -1), (-1, 0)])
    for c in range(K):
        cells = np.flatnonzero(truth == c)
        if cells.size == 0:
            continue
        want = min(per, cells.size)
        got = 0
        start = cells[rg.integers(cells.size)]
        y, x = divmod(int(start), W)
        tries = 0
        while got < want and tries < 50 * want:
            tries += 1
            p = y * W + x
            if not chosen[p]:
                chosen[p] = True
                got += 1
            if stroke_len is not None and tries % stroke_len == 0:
                start = cells[rg.integers(cells.size)]
                y, x = divmod(int(start), W)
                continue
            dy, dx = steps[rg.integers(4)]
            ny, nx = y + dy, x + dx
            if 0 <= ny < H and 0 <= nx < W and region[ny, nx] == c:
                y, x = ny, nx
            elif rg.random() < 0.02:
                start = cells[rg.integers(cells.size)]
                y, x = divmod(int(start), W)
    idx = np.flatnonzero(chosen).astype(np.int32)
    return idx, truth[idx].astype(np.int32)
