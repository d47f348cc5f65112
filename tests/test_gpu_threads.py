"""Plans used from several host threads at once, each on its own stream: plan creation,
the first factorization (recorded as a HIP graph on the plan's stream) and G(X), while
other threads do the same.  Every result must equal a one-thread run bit for bit (the
kernels are deterministic and plans share no state but the device).  This pins that no
call of the library goes through the legacy stream, which would depend on the other
threads' blocking streams and fail while one of them is being recorded."""
import sys
import threading

import numpy as np
import pytest

from paper_2310_18043_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("tile,cols", [(64, 0), (128, 0), (256, 8)])
def test_plans_on_threads_with_their_own_streams(torch_cuda, tile, cols):
    # tile 256 with eight right-hand sides per solve workgroup: the 256-thread form that
    # the batched configuration's concurrent plans run
    from paper_2310_18043_amd import rfeig
    torch = torch_cuda
    print(f"[gpu-case] plans on 8 threads, tile {tile}, trsm_cols {cols}", flush=True)
    sys.stdout.flush()
    m = 30
    A, B = W.convdiff_pencil(m, mass=(0.5, 1.5), seed=2)
    n = A.shape[0]
    c, r = (m * m * 2.0) + 0.05j, m * m * 0.8
    nthreads, rounds, ncols = 8, 2, 16
    Xs = [W.start_block(n, ncols, seed=40 + t) for t in range(nthreads)]

    def one(t, stream):
        s = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            P = rfeig.Plan(A, B, c + 3.0 * t, r, p=4, q=4, w=ncols, tile=tile, trsm_cols=cols,
                           tuned=False, stream=s)
            P.factor_shifts()
            Z = P.apply_inner(torch.from_numpy(Xs[t]).cuda())
            s.synchronize()
            out = Z.cpu().numpy()
            P.close()
        return out

    ref = [one(t, None) for t in range(nthreads)]
    got, errors = {}, []

    def worker(t):
        st = torch.cuda.Stream()
        try:
            for k in range(rounds):
                got[(t, k)] = one(t, st)
        except Exception as e:            # reported below
            errors.append((t, repr(e)))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(nthreads)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for t in range(nthreads):
        for k in range(rounds):
            assert np.array_equal(got[(t, k)], ref[t]), (t, k)
