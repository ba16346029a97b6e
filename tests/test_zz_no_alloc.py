"""The allocation-free entry point (marked gpu): oz2h_gemm_noalloc against oz2h_gemm on
two calls in a row, the second with a smaller input, and the size limit."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev_mp, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    need_gpu()
    from paper_2609_27831_amd import oz2h
    return oz2h


def _same(C1, C2):
    import torch
    return (torch.equal(C1.sign, C2.sign) and torch.equal(C1.exp, C2.exp)
            and torch.equal(C1.limbs, C2.limbs))


def test_noalloc_matches_workspace_call(oz, c_oracle):
    import torch
    calls = [(256, 300, 200, 260), (113, 70, 90, 33)]   # (p, M, N, K): second call smaller
    for i, (p, M, N, K) in enumerate(calls):
        A = synth.mp_random(900 + i, M, K, p, -16, 16)
        B = synth.mp_random(910 + i, K, N, p, -16, 16)
        plan = oz.Plan.create(p, K)
        Ad, Bd = dev_mp(A), dev_mp(B)
        out = oz.empty_mp(M, N, p)
        print(f"noalloc call {i}: p={p} M={M} N={N} K={K}", flush=True)
        C1 = oz.gemm_noalloc(plan, Ad, Bd, out=out)
        C2 = oz.gemm(plan, Ad, Bd)
        torch.cuda.synchronize()
        assert _same(C1, C2), f"call {i}"
        ref = c_oracle.gemm(A, B, want_chat=False)
        s, e, l = C1.to_host()
        assert np.array_equal(s, ref["c_sign"]) and np.array_equal(e, ref["c_exp"])
        assert np.array_equal(l, ref["c_limbs"])


def test_noalloc_size_limit(oz):
    cap = oz.lib().oz2h_gemm_noalloc_max_bytes()
    assert cap == 128 << 20
    p, K = 256, 2048
    plan = oz.Plan.create(p, K)
    M = N = 2048                                     # 1.45 GB of workspace: beyond the cap
    assert plan.workspace_size(M, N) > cap
    A = dev_mp(synth.mp_random(920, M, K, p, -4, 4))
    B = dev_mp(synth.mp_random(921, K, N, p, -4, 4))
    with pytest.raises(oz.Oz2hError) as ei:
        oz.gemm_noalloc(plan, A, B, out=oz.empty_mp(M, N, p))
    assert ei.value.code == oz.ERANGE
