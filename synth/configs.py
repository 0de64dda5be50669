"""Workload recipes.

Each recipe returns a `Problem`: a graph, the labelled node set with its labels, K and
the solver settings the workload runs with.  The recipes are stand-ins for the paper's
network and image data sets (Table 1 and Table 2 of the paper), which are not used:
every input is generated from a seed.

  sbm_small    SBM n = 1,200, three equal blocks, p_in = 0.10, p_out = 0.005, unit weights;
               5% of each class labelled; FP64; 300 iterations.
  knn_mixture  k-NN graph (k = 10, union-symmetrised) of a 10-class Gaussian mixture in
               784 dimensions, n = 70,000, locally scaled Gaussian weights; 1% labelled;
               FP32; 500 iterations.
  sbm_large    SBM n = 2,000,000, K = 5, expected degree 24, p_in / p_out = 8, unit
               weights; 0.5% labelled; FP32; 1,000 iterations.
  batch_mix    256 graphs: even index SBM (expected degree 24, ratio 8), odd index
               4-neighbour image grid; n log-uniform in [2e3, 2e5]; K uniform in 3..10;
               labelled fraction uniform in [1%, 5%]; FP32; 300 iterations.
  serve_mix    8-neighbour image grids with sides in {128, 256, 512, 1024}, K in {3, 4, 6},
               2% scribble labels; FP32; 300 iterations.

  color_image  fully connected Gaussian graph over the RGB colours of a synthetic K-region
               image (a stand-in for the paper's colour images, Table 2: n 16.5k-38.2k,
               K 4-8), sigma = 0.1 on colours in [0, 1]; 2% scribble labels; the paper's
               image setting eps = 0.1, omega0 = 1e5, one-shot.

Networks use eps = 50 and omega0 = 1000, the values the paper selects for networks in its
parameter study (Section 5.2).  The image-like grids also use eps = 50: the paper's image
setting (eps = 0.1, omega0 = 1e5) is its one-shot regime on a fully connected graph, which
on a sparse grid with few scribbles would label every unreached pixel by the lowest-index
tie rule.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import graphs


@dataclasses.dataclass
class Problem:
    graph: graphs.Graph
    labelled_idx: np.ndarray  # int32, sorted
    labels: np.ndarray        # int32 in [0, K)
    K: int
    dtype: str = "f32"        # "f32" or "f64"
    eps: float = 50.0
    omega0: float = 1000.0
    max_iter: int = 300
    tol: float = 1e-6
    name: str = ""

    @property
    def n(self) -> int:
        return self.graph.n


def sbm_small(seed: int = 0, n_per: int = 400, K: int = 3) -> Problem:
    g = graphs.sbm([n_per] * K, 0.10, 0.005, seed)
    idx, lab = graphs.stratified_labels(g.truth, K, 0.05, seed)
    return Problem(g, idx, lab, K, "f64", 50.0, 1000.0, 300, 1e-6, "sbm_small")


def knn_mixture(seed: int = 1, n: int = 70_000, d: int = 784, K: int = 10, device: str = "cpu") -> Problem:
    g = graphs.gaussian_mixture_knn(n, d, K, 10, seed, device=device)
    idx, lab = graphs.stratified_labels(g.truth, K, 0.01, seed)
    return Problem(g, idx, lab, K, "f32", 50.0, 1000.0, 500, 1e-6, "knn_mixture")


def sbm_large(seed: int = 2, n: int = 2_000_000, K: int = 5, avg_degree: float = 24.0) -> Problem:
    g = graphs.sbm_by_degree(n, K, avg_degree, 8.0, seed)
    idx, lab = graphs.stratified_labels(g.truth, K, 0.005, seed)
    return Problem(g, idx, lab, K, "f32", 50.0, 1000.0, 1000, 1e-6, "sbm_large")


def batch_member(seed: int, i: int, n_lo: float = 2e3, n_hi: float = 2e5) -> Problem:
    rg = graphs.rng_for(seed, 100 + i)
    n = int(round(math.exp(rg.uniform(math.log(n_lo), math.log(n_hi)))))
    K = int(rg.integers(3, 11))
    frac = float(rg.uniform(0.01, 0.05))
    sub = seed * 100003 + i
    if i % 2 == 0:
        g = graphs.sbm_by_degree(n, K, 24.0, 8.0, sub)
    else:
        g = graphs.image_grid(n, K, sub, neighbours=4)
    idx, lab = graphs.stratified_labels(g.truth, K, frac, sub)
    return Problem(g, idx, lab, K, "f32", 50.0, 1000.0, 300, 1e-6, f"batch[{i}]")


def batch_mix(seed: int = 3, count: int = 256, n_lo: float = 2e3, n_hi: float = 2e5) -> list:
    return [batch_member(seed, i, n_lo, n_hi) for i in range(count)]


def serve_request(seed: int, i: int, sides=(128, 256, 512, 1024), Ks=(3, 4, 6), side=None, K=None) -> Problem:
    rg = graphs.rng_for(seed, 200 + i)
    s_draw = int(sides[int(rg.integers(len(sides)))])
    k_draw = int(Ks[int(rg.integers(len(Ks)))])
    side = s_draw if side is None else int(side)
    K = k_draw if K is None else int(K)
    sub = seed * 100003 + i
    g = graphs.image_grid(side * side, K, sub, neighbours=8, side=side)
    # short strokes (4 pixels) scattered inside the regions: with a few long strokes every
    # pixel without a labelled neighbour ties at U_0 and the first step ends the solve
    idx, lab = graphs.scribble_labels(g.truth, side, side, K, 0.02, sub, stroke_len=4)
    return Problem(g, idx, lab, K, "f32", 50.0, 1000.0, 300, 1e-6, f"serve[{i}]")


def serve_pool(seed: int, sides=(128, 256, 512, 1024), Ks=(3, 4, 6), copies: int = 1) -> list:
    """`copies` requests of every (side, K) pair, each its own synthetic image and scribbles:
    drawing uniformly from this pool is drawing side and K uniformly and independently, as the
    serving mix asks."""
    pairs = [(sd, k) for k in Ks for sd in sides]
    return [serve_request(seed, c * len(pairs) + j, side=sd, K=k)
            for c in range(copies) for j, (sd, k) in enumerate(pairs)]


def lfr_many_classes(seed: int = 5, n: int = 100_000, K: int = 585, avg_degree: float = 5.0, mu: float = 0.2,
                     frac: float = 0.05, dtype: str = "f32", max_iter: int = 300) -> Problem:
    """The many-classes workload: an LFR-shaped network (power-law degrees of mean about 5,
    power-law community sizes, 20% of edge ends outside the community), K communities,
    `frac` of each community labelled, eps = 50, omega0 = 1000."""
    g = graphs.lfr_like(n, K, avg_degree, mu, seed)
    idx, lab = graphs.stratified_labels(g.truth, K, frac, seed)
    return Problem(g, idx, lab, K, dtype, 50.0, 1000.0, max_iter, 1e-6, f"lfr_many_classes(n={n},K={K})")


def grown_sbm(seed: int = 6, n_old: int = 3000, n_new: int = 150, K: int = 3, avg_degree: float = 24.0,
              frac: float = 0.05):
    """A network that grows: an SBM on n_old + n_new nodes whose first n_old nodes (in the
    randomly permuted order) are the network seen first.  Returns (old problem, grown
    problem); both label the same nodes, all of them old."""
    import numpy as np
    import scipy.sparse as sp

    g = graphs.sbm_by_degree(n_old + n_new, K, avg_degree, 8.0, seed)
    W = sp.csr_matrix((g.data, g.indices, g.indptr), shape=(g.n, g.n))
    Wo = W[:n_old, :n_old].tocsr()
    Wo.sort_indices()
    go = graphs.Graph(n_old, K, Wo.indptr.astype(np.int64), Wo.indices.astype(np.int32), Wo.data, g.truth[:n_old])
    idx, lab = graphs.stratified_labels(go.truth, K, frac, seed)
    old = Problem(go, idx, lab, K, "f64", 50.0, 1000.0, 300, 1e-6, "grown_sbm(old)")
    full = Problem(g, idx, lab, K, "f64", 50.0, 1000.0, 300, 1e-6, "grown_sbm(full)")
    return old, full


@dataclasses.dataclass
class ImageProblem:
    """A fully connected Gaussian graph given by node features (no stored edges)."""
    features: np.ndarray      # float64[n, d]
    sigma: float
    labelled_idx: np.ndarray  # int32, sorted
    labels: np.ndarray        # int32 in [0, K)
    K: int
    truth: np.ndarray         # int32[n]
    dtype: str = "f64"
    eps: float = 0.1
    omega0: float = 1e5
    max_iter: int = 300
    tol: float = 1e-6
    one_shot: bool = True
    name: str = ""

    @property
    def n(self) -> int:
        return self.features.shape[0]


def color_image(seed: int = 7, H: int = 196, W: int = 195, K: int = 4, sigma: float = 0.1, frac: float = 0.02,
                dtype: str = "f64") -> ImageProblem:
    """The image workload: a synthetic H x W colour image of K regions (196 x 195 = 38,220
    pixels, K = 4: the size of the largest image of Table 2), its pixels the nodes of a fully
    connected Gaussian graph on their colours, scribbles on 2% of the pixels."""
    feats, truth = graphs.color_image(H, W, K, seed)
    idx, lab = graphs.scribble_labels(truth, H, W, K, frac, seed, stroke_len=8)
    return ImageProblem(feats, sigma, idx, lab, K, truth, dtype, name=f"color_image({H}x{W},K={K})")
