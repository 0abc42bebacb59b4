"""Vector quantisation of editable Gaussians (Sec. 4.4) and composition of
quantised models (Sec. 4.5), plain numpy.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
CPU-baseline leg, never by the product path; it shares no code with the HIP
library.

What the paper fixes: k-means gives one codebook per attribute over all the
Gaussians of a basic model; a vector attribute shares one scalar codebook,
with a separate index per component; mean and normal stay exact; the other
attributes are rotation q, scale s, opacity o, offset colour delta-c and the
shading terms k_a, k_d, k_s, beta (Sec. 4.3), so eight codebooks.  Readings
where it is silent (the same on the GPU side):
  - codebook size k <= 256 (one byte per index), chosen by the caller;
  - initial centroids at the centres of k equal cells of [min, max] of the
    finite values, in FP32: lo + (j + 1/2) * ((hi - lo) / k);
  - Lloyd iterations, a caller-chosen count: assign every value to its
    nearest centroid (|x - c| in FP32, the lowest index on ties), then each
    centroid becomes the FP64 mean of its values rounded to FP32 (an empty
    cluster keeps its centroid), then the codebook is sorted ascending;
  - the stored indices are the assignment to the final codebook;
  - non-finite values take index 0 and do not move any centroid.
"""
from __future__ import annotations

import numpy as np

# Codebooks of a quantised model and the 15 index planes, in the order of
# the float planes log_scale (3), quat (4), opacity (1), color (3), shade (4).
CODEBOOKS = ("log_scale", "quat", "opacity", "color", "k_a", "k_d", "k_s", "beta")
PLANE_BOOK = (0, 0, 0, 1, 1, 1, 1, 2, 3, 3, 3, 4, 5, 6, 7)
INDEX_PLANES = (("log_scale", 3), ("quat", 4), ("opacity", 1), ("color", 3), ("shade", 4))

_BLOCK = 1 << 16  # values per block of the brute-force assignment


def assign(values, codebook) -> np.ndarray:
    """Nearest centroid of each value by brute force over the whole codebook:
    argmin_j |x - c_j| with the difference taken in FP32 (the first index on
    ties); non-finite values take 0.  uint8 indices (k <= 256)."""
    x = np.asarray(values, np.float32).ravel()
    c = np.asarray(codebook, np.float32).ravel()
    out = np.zeros(x.size, np.uint8)
    for b in range(0, x.size, _BLOCK):
        xb = x[b:b + _BLOCK]
        d = np.abs(xb[:, None] - c[None, :])  # float32 - float32: correctly rounded
        out[b:b + _BLOCK] = np.argmin(d, axis=1)
    out[~np.isfinite(x)] = 0
    return out


def init_codebook(values, k: int) -> np.ndarray:
    """Centres of k equal cells of [min, max] over the finite values, in FP32;
    all zero when no value is finite."""
    x = np.asarray(values, np.float32).ravel()
    x = x[np.isfinite(x)]
    if x.size == 0:
        return np.zeros(k, np.float32)
    lo, hi = np.float32(x.min()), np.float32(x.max())
    w = np.float32(np.float32(hi - lo) / np.float32(k))
    j = np.arange(k, dtype=np.float32)
    return (lo + (j + np.float32(0.5)) * w).astype(np.float32)


def lloyd_step(values, codebook) -> np.ndarray:
    """One Lloyd iteration: assign, move each non-empty cluster's centroid to
    the FP64 mean of its values (rounded to FP32), sort ascending."""
    x = np.asarray(values, np.float32).ravel()
    c = np.asarray(codebook, np.float32).ravel()
    idx = assign(x, c)
    ok = np.isfinite(x)
    sums = np.bincount(idx[ok], weights=x[ok].astype(np.float64), minlength=c.size)
    counts = np.bincount(idx[ok], minlength=c.size)
    new = c.copy()
    nz = counts > 0
    new[nz] = (sums[nz] / counts[nz]).astype(np.float32)
    return np.sort(new, kind="stable")


def fit(values, k: int, iters: int):
    """k-means codebook of one attribute and the indices of its values."""
    c = init_codebook(values, k)
    for _ in range(iters):
        c = lloyd_step(values, c)
    return c, assign(values, c)


def objective(values, codebook, index) -> float:
    """Sum of squared quantisation errors over the finite values, FP64."""
    x = np.asarray(values, np.float64).ravel()
    ok = np.isfinite(x)
    q = np.asarray(codebook, np.float64)[np.asarray(index).ravel()]
    return float(((x - q)[ok] ** 2).sum())


def quantize(planes: dict, k: int, iters: int) -> dict:
    """Quantised form of one basic model: exact mean and normal, eight
    codebooks [8, k] and the 15 index planes [15, n] (uint8)."""
    n = planes["mean"].shape[1]
    rows = np.concatenate([np.asarray(planes[name], np.float32).reshape(d, n) for name, d in INDEX_PLANES])
    books = np.zeros((len(CODEBOOKS), k), np.float32)
    index = np.zeros((15, n), np.uint8)
    for b in range(len(CODEBOOKS)):
        sel = [p for p in range(15) if PLANE_BOOK[p] == b]
        c, idx = fit(rows[sel].ravel(), k, iters)  # components concatenated: one shared codebook
        books[b] = c
        index[sel] = idx.reshape(len(sel), n)
    return {"mean": np.asarray(planes["mean"], np.float32), "normal": np.asarray(planes["normal"], np.float32),
            "codebook": books, "index": index}


def decode(q: dict) -> dict:
    """The float planes of a quantised model: each index plane reads its
    codebook; mean and normal as stored."""
    books, index = q["codebook"], q["index"]
    rows = np.stack([books[PLANE_BOOK[p]][index[p]] for p in range(15)]).astype(np.float32)
    out = {"mean": q["mean"], "normal": q["normal"]}
    r = 0
    for name, d in INDEX_PLANES:
        out[name] = np.ascontiguousarray(rows[r:r + d])
        r += d
    return out
