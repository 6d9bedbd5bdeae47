"""The integer step thresholds the kernels bin by against the direct binary64 classification of
N = k dN (Sec. 2.1; bins are right-closed, N in (e_j, e_{j+1}]) that the oracle uses, for every
step count up to the cap, including edges that sit exactly on some fl(k dN)."""
import ctypes

import numpy as np
import pytest

import oracle as O


def _thresholds(lib, edges, dN):
    edges = np.ascontiguousarray(edges, np.float64)
    out = np.zeros(len(edges), np.uint32)
    rc = lib.load().pyfpt_bin_thresholds(ctypes.c_void_p(edges.ctypes.data), len(edges), float(dN),
                                         ctypes.c_void_p(out.ctypes.data))
    assert rc == 0
    return out


def _rows_from_thresholds(K, k):
    """Row of a run of k steps by the kernels' rule: bin j when K_j < k <= K_{j+1}, B below the
    range (k <= K_0), B + 1 above it (k > K_B)."""
    B = len(K) - 1
    lo = np.searchsorted(K.astype(np.int64), k.astype(np.int64), side="left")   # first K >= k
    return np.where(lo == 0, B, np.where(lo == B + 1, B + 1, lo - 1))


@pytest.fixture(scope="module")
def lib():
    from paper_2206_11234_amd import _lib
    return _lib


@pytest.mark.parametrize("dN,n_bins,seed", [(1e-3, 100, 0), (5e-4, 200, 1), (1e-4, 500, 2), (0.1, 37, 3)])
def test_thresholds_match_binary64_classification(lib, dN, n_bins, seed):
    rng = np.random.default_rng(seed)
    k_max = 200_000
    top = k_max * dN
    edges = np.sort(rng.uniform(0.0, top, n_bins + 1))
    # put a third of the edges exactly on a product fl(k dN), the boundary case of a right-closed bin
    on = rng.choice(n_bins + 1, (n_bins + 1) // 3, replace=False)
    edges[on] = rng.integers(1, k_max, on.size).astype(np.float64) * dN
    edges = np.unique(edges)
    K = _thresholds(lib, edges, dN)
    k = np.arange(k_max + 1, dtype=np.uint64)
    want = O.bin_rows(k, np.full(k.size, O.ST_ENDED, np.int32), dN, edges)
    assert np.array_equal(_rows_from_thresholds(K, k), want)


def test_thresholds_clamp_and_reject(lib):
    K = _thresholds(lib, np.array([-1.0, 0.0, 1e30]), 1e-3)
    assert K[0] == 0 and K[1] == 0 and K[2] == 0xFFFFFFFF
    out = np.zeros(1, np.uint32)
    e = np.zeros(1)
    assert lib.load().pyfpt_bin_thresholds(ctypes.c_void_p(e.ctypes.data), 1, 0.0,
                                           ctypes.c_void_p(out.ctypes.data)) == lib.PYFPT_EINVAL
