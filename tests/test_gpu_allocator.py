"""Device memory through the caller's allocator (rf_allocator, include/rfeig.h).

The boundary of Alg. composite's REQUIRE/ENSURE: the plan owns its factors, Krylov
basis and scratch, but every byte of them comes from the caller's callbacks, so that
PyTorch's caching allocator supplies all device memory.  Through the C ABI.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_2310_18043_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def rf(torch_cuda):
    from paper_2310_18043_amd import rfeig
    return rfeig


class CountingAllocator:
    """Callbacks that take memory from torch's caching allocator and keep count of
    every pointer handed out and returned.  fail_after: refuse the n-th request."""

    def __init__(self, rf, torch, fail_after=None):
        self.rf, self.torch = rf, torch
        self.live, self.calls, self.frees, self.total = {}, 0, 0, 0
        self.fail_after = fail_after

        def _alloc(nbytes, ctx):
            self.calls += 1
            if self.fail_after is not None and self.calls > self.fail_after:
                return None
            ptr = int(torch.cuda.caching_allocator_alloc(int(nbytes)))
            self.live[ptr] = int(nbytes)
            self.total += int(nbytes)
            return ptr

        def _free(ptr, ctx):
            self.frees += 1
            assert int(ptr) in self.live, "freed a pointer the allocator never gave out"
            del self.live[int(ptr)]
            torch.cuda.caching_allocator_delete(int(ptr))

        self._a, self._f = rf.ALLOC_FN(_alloc), rf.FREE_FN(_free)
        self.struct = rf.RfAllocator(self._a, self._f, None)


def _small_pencil():
    A, B = W.convdiff_pencil(20, mass=(0.5, 1.5), seed=1)      # N = 400, kl = 20
    return A, B, 900 + 0.05j, 250.0


def test_plan_memory_is_torch_memory(rf, torch_cuda):
    A, B, c, r = _small_pencil()
    torch_cuda.cuda.synchronize()
    base = torch_cuda.cuda.memory_allocated()
    _say("plan with the torch caching allocator")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=16)
    held = torch_cuda.cuda.memory_allocated() - base
    print("plan device bytes", plan.device_bytes, "torch memory_allocated delta", held)
    assert plan.device_bytes > 0
    # every plan buffer is a torch block (the caching allocator rounds sizes up)
    assert held >= plan.device_bytes
    assert plan.allocator.live_bytes == plan.device_bytes
    plan.factor_shifts()
    plan.close()
    torch_cuda.cuda.synchronize()
    assert torch_cuda.cuda.memory_allocated() == base


def test_counting_allocator_sees_every_byte_and_gets_all_back(rf, torch_cuda):
    from oracle import filters
    A, B, c, r = _small_pencil()
    alloc = CountingAllocator(rf, torch_cuda)
    _say("plan with a counting allocator")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=16, allocator=alloc)
    assert alloc.total == plan.device_bytes and alloc.calls == len(alloc.live)
    plan.factor_shifts()
    X = W.start_block(A.shape[0], 16, seed=2)
    Z = plan.apply_inner(torch_cuda.from_numpy(X).cuda()).cpu().numpy()
    ref = filters.InnerOperator(A, B, c, r, 4)(X)
    assert np.linalg.norm(Z - ref) / np.linalg.norm(ref) <= 1e-12
    # the same plan on hipMalloc memory gives the same numbers bit for bit
    plain = rf.Plan(A, B, c, r, p=4, q=8, w=16, allocator=None)
    plain.factor_shifts()
    Z2 = plain.apply_inner(torch_cuda.from_numpy(X).cuda()).cpu().numpy()
    assert np.array_equal(Z, Z2)
    plain.close()
    plan.close()
    assert not alloc.live and alloc.frees == alloc.calls


def test_adjoint_plan_uses_the_same_allocator(rf, torch_cuda):
    A, B, c, r = _small_pencil()
    alloc = CountingAllocator(rf, torch_cuda)
    _say("adjoint plan with a counting allocator")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=16, allocator=alloc)
    n1 = alloc.calls
    adj = plan.adjoint()
    assert alloc.calls > n1 and alloc.total == plan.device_bytes + adj.device_bytes
    adj.close()
    plan.close()
    assert not alloc.live


def test_batch_memory_through_the_allocator(rf, torch_cuda):
    A, B = W.convdiff_pencil(16, mass=None)
    alloc = CountingAllocator(rf, torch_cuda)
    disks = [dict(c=400 + 0.05j, r=120.0, p=4, q=4, w=8), dict(c=900 + 0.05j, r=150.0, p=2, q=8, w=16)]
    _say("batch of 2 disks with a counting allocator")
    bt = rf.Batch(A, B, disks, allocator=alloc)
    assert alloc.total == bt.device_bytes
    bt.factor()
    bt.close()
    assert not alloc.live and alloc.frees == alloc.calls


def test_allocator_failure_is_reported_and_nothing_leaks(rf, torch_cuda):
    A, B, c, r = _small_pencil()
    alloc = CountingAllocator(rf, torch_cuda, fail_after=10)
    _say("plan whose allocator refuses the 11th request")
    with pytest.raises(rf.RfError) as ei:
        rf.Plan(A, B, c, r, p=4, q=8, w=16, allocator=alloc)
    assert ei.value.status == rf.RF_ERR_NOMEM
    assert "allocator" in str(ei.value)
    assert not alloc.live and alloc.frees == 10
