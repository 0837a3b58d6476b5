"""CPU tests of the binding's argument checks: host tensors passed as device
memory and mis-sized outputs are rejected with ValueError before any
allocation or library call (the C ABI only sees pointers)."""
import ctypes

import pytest
import torch

import paper_1405_2912_amd as ftv


class Dev:
    """A stand-in for a device tensor: only the attributes the checks read."""

    def __init__(self, numel, dtype=torch.float32, device="cuda:0", contiguous=True):
        self._n = numel
        self.dtype = dtype
        self.device = torch.device(device)
        self.is_cuda = self.device.type == "cuda"
        self._c = contiguous

    def numel(self):
        return self._n

    def element_size(self):
        return torch.empty(0, dtype=self.dtype).element_size()

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        raise AssertionError("a rejected call must not reach the library")


class NoCtx:
    @property
    def handle(self):
        raise AssertionError("a rejected call must not reach the library")


def _raises(fn, match):
    with pytest.raises(ValueError, match=match):
        fn()


def test_host_tensors_are_not_device_memory():
    x = torch.zeros(16)
    _raises(lambda: ftv.vote(NoCtx(), [x, x, x], ftv.ulp(4)), "CUDA")
    _raises(lambda: ftv.vote_blocks(NoCtx(), [x, x, x], ftv.exact(), 4096), "CUDA")
    _raises(lambda: ftv.fingerprint(NoCtx(), x, 4096), "CUDA")
    _raises(lambda: ftv.make_desc([x, x], ftv.exact()), "CUDA")
    d = Dev(16)
    _raises(lambda: ftv.vote(NoCtx(), [d, d, d], ftv.ulp(4), consensus=torch.zeros(16)), "consensus")


def test_replicas_must_match():
    a, b = Dev(100), Dev(99)
    _raises(lambda: ftv.vote(NoCtx(), [a, b, a], ftv.ulp(4)), "replica 1 has 99")
    c = Dev(100, dtype=torch.float64)
    _raises(lambda: ftv.vote(NoCtx(), [a, c], ftv.ulp(4)), "dtype")
    e = Dev(100, device="cuda:1")
    _raises(lambda: ftv.vote(NoCtx(), [a, e], ftv.ulp(4)), "cuda:1")
    _raises(lambda: ftv.vote(NoCtx(), [a, Dev(100, contiguous=False)], ftv.ulp(4)), "contiguous")
    _raises(lambda: ftv.vote(NoCtx(), [a] * 8, ftv.ulp(4)), "at most 7")
    _raises(lambda: ftv.make_desc([a, a], ftv.exact(), n=101), "needs at least 101")


def test_outputs_must_be_large_enough():
    a = Dev(1000)
    _raises(lambda: ftv.vote(NoCtx(), [a, a, a], ftv.ulp(4), consensus=Dev(999)), "consensus")
    _raises(lambda: ftv.vote(NoCtx(), [a, a, a], ftv.ulp(4), consensus=Dev(1000, torch.int32)), "consensus")
    _raises(lambda: ftv.vote(NoCtx(), [a, a, a], ftv.ulp(4), mask=Dev(999, torch.uint8)), "mask")
    _raises(lambda: ftv.vote(NoCtx(), [a, a, a], ftv.ulp(4), mask=Dev(1000, torch.int8)), "mask")
    small_stats = Dev(ctypes.sizeof(ftv.Stats) // 8 - 1, torch.int64)
    _raises(lambda: ftv.vote(NoCtx(), [a, a, a], ftv.ulp(4), stats=small_stats), "stats")
    _raises(lambda: ftv.make_desc([a, a], ftv.exact(), None, None, small_stats), "stats")


def test_block_and_fingerprint_outputs():
    a = Dev(3 * 8192, torch.float64)       # 3 blocks of 64 KiB
    _raises(lambda: ftv.vote_blocks(NoCtx(), [a, a, a], ftv.exact(), 65536, fps=Dev(8, torch.int64)), "fps")
    _raises(lambda: ftv.vote_blocks(NoCtx(), [a, a, a], ftv.exact(), 65536, blockmap=Dev(2, torch.uint8)),
            "blockmap")
    _raises(lambda: ftv.vote_blocks(NoCtx(), [a, a, a], ftv.exact(), 65536, bstats=Dev(3, torch.int64)),
            "bstats")
    _raises(lambda: ftv.vote_blocks(NoCtx(), [a, a, a], ftv.exact(), 65536, mask=Dev(10, torch.uint8)), "mask")
    _raises(lambda: ftv.fingerprint(NoCtx(), a, 65536, out=Dev(2, torch.int64)), "fingerprint output")


def test_vote_mem_takes_host_replicas_but_device_outputs():
    a = Dev(64)
    h = torch.zeros(64)
    _raises(lambda: ftv.vote_mem(NoCtx(), [a, h], ftv.ulp(4), consensus=torch.zeros(64)), "consensus")
    _raises(lambda: ftv.vote_mem(NoCtx(), [a, torch.zeros(63)], ftv.ulp(4)), "replica 1 has 63")


def test_vote_host_rejects_bad_arrays():
    import numpy as np
    a = np.zeros(100, dtype=np.float32)
    with pytest.raises(ValueError):
        ftv.vote_host([a, a[::2], a], ftv.ulp(4))                # not contiguous
    with pytest.raises(ValueError):
        ftv.vote_host([a, a.astype(np.float64), a], ftv.ulp(4))  # mixed dtypes
    with pytest.raises(ValueError):
        ftv.vote_host([a, a[:50], a], ftv.ulp(4))                # a replica too short
    with pytest.raises(ValueError):
        ftv.vote_host([a.astype(np.float16)] * 3, ftv.ulp(4))    # unsupported dtype
    with pytest.raises(ValueError):
        ftv.vote_host([a] * 8, ftv.ulp(4))                       # more than 7 replicas


def test_vote_placed_rejects_outputs_in_the_wrong_memory():
    a = torch.zeros(16)
    with pytest.raises(ValueError):
        ftv.vote_placed(NoCtx(), None, [a, a, a], ftv.ulp(4), out_memory=ftv.MEM_DEVICE,
                        consensus=torch.zeros(16))               # a host tensor as device output
