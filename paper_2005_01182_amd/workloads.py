"""Seeded synthetic inputs for the assignment and transport workloads.

This module only builds inputs: integer cost matrices, integer masses and
request traces.  It contains none of the solver's arithmetic, and both the
CPU oracle tests and the GPU path read the arrays it returns.

The workloads stand in for the paper's data sets (Section 3.2, Table 1), which
are not redistributed here:

* ``uniform_assignment``    -- i.i.d. integer costs, the small plain-KM case.
* ``geometric_assignment``  -- noisy circle vs. noisy square perimeter, the
  CircleSquare family (Section 3.2), Euclidean cost scaled by 1e4.
* ``pixel_histogram_pair``  -- two 28x28 blob images with integer mass, the
  MNIST family (Section 3.2; Table 1 rows mnist0-9), squared grid distance.
* ``embedding_batch``       -- many uneven assignment problems between sets of
  300-d vectors with near-duplicates, the NLP family in spirit (Section 3.2).
* ``serving_trace`` / ``grid_points_cost`` -- Poisson request stream whose
  costs are rounded Euclidean distances between integer grid points.
* ``knn_graph`` / ``knn_assignment`` -- sparse cost graphs in CSR: each source
  point keeps its k nearest targets (plus, optionally, one edge of a random
  perfect matching so that every row can be matched), the sparse form of the
  geometric family.

Every generator is a pure function of its seed (numpy PCG64; independent
sub-streams come from ``SeedSequence(seed).spawn``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for",
    "uniform_assignment",
    "geometric_points",
    "geometric_assignment",
    "blob_image",
    "largest_remainder",
    "pixel_histogram",
    "grid_sq_cost",
    "pixel_histogram_pair",
    "embedding_sizes",
    "embedding_problem",
    "embedding_batch",
    "isqrt_round",
    "grid_points_cost",
    "ServingRequest",
    "serving_trace",
    "knn_graph",
    "knn_assignment",
    "knn_batch",
    "csr_to_dense",
]


def rng_for(seed: int, k: int | None = None):
    """PCG64 generator for ``seed``; with ``k`` return ``k`` independent children."""
    if k is None:
        return np.random.Generator(np.random.PCG64(seed))
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(k)]


# --------------------------------------------------------------------------- #
# Uniform integer costs (small plain case)
# --------------------------------------------------------------------------- #
def uniform_assignment(n: int = 64, lo: int = 0, hi: int = 1000, seed: int = 0) -> np.ndarray:
    """n x n int32 costs, i.i.d. uniform integers in [lo, hi] (inclusive), row-major draw order."""
    return rng_for(seed).integers(lo, hi, endpoint=True, size=(n, n)).astype(np.int32)


# --------------------------------------------------------------------------- #
# Geometric: circle vs. square perimeter (CircleSquare family)
# --------------------------------------------------------------------------- #
def geometric_points(n: int, seed: int = 0, sigma: float = 0.02, m: int | None = None):
    """Sources on the unit circle, targets on the perimeter of the side-1 square.

    Both shapes share the origin as centre (as in the CircleSquare data).
    Sources: angle ~ U[0, 2 pi).  Targets: arclength t ~ U[0, 4) walked
    counter-clockwise from (-1/2, -1/2).  Both get N(0, sigma^2) noise per
    coordinate.  Returns (n, 2) sources and (m, 2) targets (m = n by default),
    float64; the targets' stream is independent of n.
    """
    m = n if m is None else m
    ra, rb = rng_for(seed, 2)
    th = ra.uniform(0.0, 2.0 * np.pi, n)
    x = np.stack([np.cos(th), np.sin(th)], axis=1) + ra.normal(0.0, sigma, (n, 2))
    t = rb.uniform(0.0, 4.0, m)
    side = np.minimum(np.floor(t).astype(np.int64), 3)
    f = t - side
    y = np.empty((m, 2))
    s0, s1, s2, s3 = (side == 0), (side == 1), (side == 2), (side == 3)
    y[s0, 0], y[s0, 1] = -0.5 + f[s0], -0.5
    y[s1, 0], y[s1, 1] = 0.5, -0.5 + f[s1]
    y[s2, 0], y[s2, 1] = 0.5 - f[s2], 0.5
    y[s3, 0], y[s3, 1] = -0.5, 0.5 - f[s3]
    y += rb.normal(0.0, sigma, (m, 2))
    return x, y


def _euclid_rint(x: np.ndarray, y: np.ndarray, scale: float) -> np.ndarray:
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(-1))
    return np.rint(scale * d).astype(np.int32)


def geometric_assignment(n: int = 2048, seed: int = 0, scale: float = 1e4) -> np.ndarray:
    """n x n int32 costs C_ij = rint(scale * ||x_i - y_j||_2) (round half to even, fp64)."""
    x, y = geometric_points(n, seed)
    return _euclid_rint(x, y, scale)


def geometric_rect(n: int, m: int, seed: int = 0, scale: float = 1e4) -> np.ndarray:
    """n x m int32 costs between n circle points and m square-perimeter points
    (rectangular CircleSquare), C_ij = rint(scale * ||x_i - y_j||_2)."""
    x, y = geometric_points(n, seed, m=m)
    return _euclid_rint(x, y, scale)


# --------------------------------------------------------------------------- #
# Pixel histograms (MNIST family)
# --------------------------------------------------------------------------- #
def blob_image(side: int = 28, seed: int = 0) -> np.ndarray:
    """Smoothed Gaussian-blob image, float64 (side, side), indexed [y, x].

    k ~ U{3..6} blobs; centre ~ U[0, side-1]^2; sigma ~ U[1, 3] px;
    amplitude ~ U[0.5, 1].
    """
    rng = rng_for(seed)
    k = int(rng.integers(3, 6, endpoint=True))
    ys, xs = np.mgrid[0:side, 0:side].astype(np.float64)
    img = np.zeros((side, side))
    for _ in range(k):
        cx, cy = rng.uniform(0.0, side - 1, 2)
        sg = rng.uniform(1.0, 3.0)
        a = rng.uniform(0.5, 1.0)
        img += a * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2.0 * sg * sg))
    return img


def largest_remainder(w: np.ndarray, total: int) -> np.ndarray:
    """Integer vector summing exactly to ``total``, proportional to ``w`` >= 0.

    Floors of the proportional shares, then +1 to the largest fractional parts
    (ties -> lowest index).  Zero weights stay zero.
    """
    w = np.asarray(w, dtype=np.float64)
    s = w.sum()
    if s <= 0:
        raise ValueError("weights must have a positive sum")
    share = w * (total / s)
    base = np.floor(share).astype(np.int64)
    rem = int(total - base.sum())
    frac = share - base
    frac[w <= 0] = -1.0
    order = np.lexsort((np.arange(len(w)), -frac))
    base[order[:rem]] += 1
    return base


def pixel_histogram(side: int = 28, seed: int = 0, zero_frac: float = 0.6, total: int = 1024) -> np.ndarray:
    """Integer mass per bin (bin k = side*y + x), int32, sums to ``total``.

    The ``round(zero_frac * side^2)`` smallest bins are zeroed first (ties ->
    lower index), then the rest is scaled to ``total`` by largest remainder.
    """
    img = blob_image(side, seed).reshape(-1)
    nz = int(round(zero_frac * img.size))
    order = np.lexsort((np.arange(img.size), img))
    w = img.copy()
    w[order[:nz]] = 0.0
    return largest_remainder(w, total).astype(np.int32)


def grid_sq_cost(side: int = 28) -> np.ndarray:
    """C[k, l] = (x_k - x_l)^2 + (y_k - y_l)^2 on a side x side grid, int32."""
    k = np.arange(side * side)
    x, y = k % side, k // side
    return ((x[:, None] - x[None, :]) ** 2 + (y[:, None] - y[None, :]) ** 2).astype(np.int32)


def pixel_histogram_pair(side: int = 28, seeds=(0, 1), total: int = 1024):
    """(C, r, c) for the pixel-histogram transport workload; zero bins included."""
    r = pixel_histogram(side, seeds[0], total=total)
    c = pixel_histogram(side, seeds[1], total=total)
    return grid_sq_cost(side), r, c


# --------------------------------------------------------------------------- #
# Batched embeddings (NLP family in spirit)
# --------------------------------------------------------------------------- #
def embedding_sizes(count: int = 4096, lo: int = 16, hi: int = 512, seed: int = 0) -> np.ndarray:
    """Problem sizes n_k ~ U{lo..hi}, int32."""
    return rng_for(seed, 1)[0].integers(lo, hi, endpoint=True, size=count).astype(np.int32)


def _with_near_duplicates(rng, n: int, dim: int, frac: float, noise: float) -> np.ndarray:
    x = rng.normal(0.0, 1.0, (n, dim))
    k = int(math.floor(frac * n))
    if k > 0 and n > 1:
        dst = rng.choice(n, size=k, replace=False)
        for d in dst:
            src = int(rng.integers(0, n - 1))
            src = src + 1 if src >= d else src  # another row of the same side
            x[d] = x[src] + rng.normal(0.0, noise, dim)
    return x


def embedding_problem(n: int, seed: int, k: int, dim: int = 300, scale: float = 1e3,
                      dup_frac: float = 0.1, noise: float = 0.1) -> np.ndarray:
    """Problem ``k`` of the embedding batch: C = rint(scale * ||x - y||_2), int32.

    Each side holds n i.i.d. N(0, 1) vectors in R^dim; on each side
    floor(dup_frac * n) rows are replaced by a copy of another row of the same
    side plus N(0, noise^2) noise.
    """
    ss = np.random.SeedSequence([seed, 1, k])
    rx, ry = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(2)]
    x = _with_near_duplicates(rx, n, dim, dup_frac, noise)
    y = _with_near_duplicates(ry, n, dim, dup_frac, noise)
    sq = (x * x).sum(1)[:, None] + (y * y).sum(1)[None, :] - 2.0 * (x @ y.T)
    return np.rint(scale * np.sqrt(np.maximum(sq, 0.0))).astype(np.int32)


def embedding_batch(count: int = 4096, lo: int = 16, hi: int = 512, seed: int = 0, dim: int = 300):
    """List of ``count`` int32 cost matrices with sizes from ``embedding_sizes``."""
    sizes = embedding_sizes(count, lo, hi, seed)
    return [embedding_problem(int(n), seed, k, dim) for k, n in enumerate(sizes)]


# --------------------------------------------------------------------------- #
# Serving stream: integer grid points, exactly rounded Euclidean cost
# --------------------------------------------------------------------------- #
def isqrt_round(d: np.ndarray) -> np.ndarray:
    """round(sqrt(d)) for int64 d >= 0, exact (no ties: sqrt(d) is never k + 1/2).

    k = floor(sqrt(d)); result k + 1 when d - k^2 > k.
    """
    d = np.asarray(d, dtype=np.int64)
    k = np.floor(np.sqrt(d.astype(np.float64))).astype(np.int64)
    # correct the float estimate to the exact integer floor
    k = np.where(k * k > d, k - 1, k)
    k = np.where((k + 1) * (k + 1) <= d, k + 1, k)
    return k + ((d - k * k) > k)


def grid_points_cost(ps: np.ndarray, pt: np.ndarray) -> np.ndarray:
    """C_ij = round(sqrt(|p_i - q_j|^2)) for integer points (n, 2), int32."""
    ps = np.asarray(ps, dtype=np.int64)
    pt = np.asarray(pt, dtype=np.int64)
    dx = ps[:, None, 0] - pt[None, :, 0]
    dy = ps[:, None, 1] - pt[None, :, 1]
    return isqrt_round(dx * dx + dy * dy).astype(np.int32)


@dataclass
class ServingRequest:
    rid: int
    t_arrival: float      # seconds from stream start
    n: int
    src: np.ndarray       # (n, 2) int32 grid points
    dst: np.ndarray       # (n, 2) int32 grid points


def serving_trace(rate: float = 2000.0, duration: float = 60.0, lo: int = 32, hi: int = 4096,
                  grid: int = 10000, seed: int = 0, limit: int | None = None):
    """Open-loop Poisson request stream.

    Inter-arrival ~ Exp(rate); n = round(exp(U[ln lo, ln hi])); points
    ~ U[0, 1]^2 quantised to p = rint(grid * x).  Generated lazily so a long
    trace never sits in memory at once.
    """
    rng_t, rng_n, rng_p = rng_for(seed, 3)
    t = 0.0
    rid = 0
    while True:
        t += rng_t.exponential(1.0 / rate)
        if t >= duration or (limit is not None and rid >= limit):
            return
        n = int(round(math.exp(rng_n.uniform(math.log(lo), math.log(hi)))))
        src = np.rint(grid * rng_p.uniform(0.0, 1.0, (n, 2))).astype(np.int32)
        dst = np.rint(grid * rng_p.uniform(0.0, 1.0, (n, 2))).astype(np.int32)
        yield ServingRequest(rid, t, n, src, dst)
        rid += 1


# --------------------------------------------------------------------------- #
# Sparse cost graphs (k nearest neighbours, CSR)
# --------------------------------------------------------------------------- #
def knn_graph(ps: np.ndarray, pt: np.ndarray, k: int, extra=None, chunk: int = 1024):
    """CSR graph from source points ps (n, 2) to target points pt (m, 2), integer.

    Row i keeps the k targets nearest to ps[i] (squared distance, ties to the
    smaller index) and, when ``extra`` is given, also column extra[i]; the edge
    cost is round(|p - q|) (as ``grid_points_cost``).  Columns are sorted within
    each row.  Returns (ptr int64[n + 1], idx int32[nnz], cost int32[nnz]).
    """
    ps = np.asarray(ps, dtype=np.int64)
    pt = np.asarray(pt, dtype=np.int64)
    n, m = ps.shape[0], pt.shape[0]
    k = min(int(k), m)
    rows = []
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        dx = ps[a:b, None, 0] - pt[None, :, 0]
        dy = ps[a:b, None, 1] - pt[None, :, 1]
        d2 = dx * dx + dy * dy
        # exact k smallest with ties to the smaller column: sort by (d2, column)
        key = d2 * m + np.arange(m)[None, :]
        near = np.argpartition(key, k - 1, axis=1)[:, :k] if k < m else np.tile(np.arange(m), (b - a, 1))
        rows.append(near)
    near = np.concatenate(rows, axis=0) if rows else np.zeros((0, k), np.int64)
    ptr = np.zeros(n + 1, np.int64)
    idx_l, cst_l = [], []
    for i in range(n):
        cols = set(int(j) for j in near[i])
        if extra is not None:
            cols.add(int(extra[i]))
        cols = np.array(sorted(cols), np.int64)
        d = pt[cols] - ps[i]
        idx_l.append(cols.astype(np.int32))
        cst_l.append(isqrt_round((d * d).sum(1)).astype(np.int32))
        ptr[i + 1] = ptr[i] + cols.size
    idx = np.concatenate(idx_l) if idx_l else np.zeros(0, np.int32)
    cst = np.concatenate(cst_l) if cst_l else np.zeros(0, np.int32)
    return ptr, idx, cst


def knn_assignment(n: int, m: int | None = None, k: int = 16, grid: int = 10000, matchable: bool = True,
                   seed: int = 0):
    """Sparse assignment instance: n source and m >= n target points ~ U{0..grid}^2,
    each source joined to its k nearest targets; with ``matchable`` every row also
    gets the edge to its partner in a random injective map, so some matching
    covers all rows.  Returns (ptr, idx, cost, n, m)."""
    m = n if m is None else int(m)
    rng_p, rng_x = rng_for(seed, 2)
    ps = rng_p.integers(0, grid, size=(n, 2), endpoint=True)
    pt = rng_p.integers(0, grid, size=(m, 2), endpoint=True)
    extra = rng_x.permutation(m)[:n] if matchable else None
    ptr, idx, cst = knn_graph(ps, pt, k, extra)
    return ptr, idx, cst, n, m


def knn_batch(count: int = 4096, lo: int = 16, hi: int = 512, k: int = 16, seed: int = 0):
    """``count`` matchable k-NN instances with n ~ U{lo..hi} (square)."""
    sizes = embedding_sizes(count, lo, hi, seed)
    return [knn_assignment(int(n), k=k, seed=seed * 1000003 + j) for j, n in enumerate(sizes)]


def csr_to_dense(ptr, idx, cst, n: int, m: int, missing: int) -> np.ndarray:
    """Dense n x m int32 matrix of the graph's costs with ``missing`` where no edge is."""
    C = np.full((n, m), missing, np.int32)
    rows = np.repeat(np.arange(n), np.diff(np.asarray(ptr, np.int64)))
    C[rows, np.asarray(idx, np.int64)] = cst
    return C
