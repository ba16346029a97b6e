"""Operand reuse through residue handles (marked gpu).

A product from saved residues (oz2h_gemm_from_residues) must equal the plain call on
the same operands bit for bit, for several right-hand (or left-hand) sides, and the
oracle on the same inputs.
"""
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


def _vs_oracle(C, A, B, c_oracle):
    ref = c_oracle.gemm(A, B, want_chat=False)
    s, e, l = C.to_host()
    assert np.array_equal(s, ref["c_sign"]) and np.array_equal(e, ref["c_exp"])
    assert np.array_equal(l, ref["c_limbs"])


@pytest.mark.parametrize("p,M,K,Ns,opA", [(256, 200, 300, (130, 77, 256), 0),
                                          (113, 129, 1000, (64, 300), 1),
                                          (2048, 40, 70, (33, 50), 0)])
def test_reuse_left_operand(oz, c_oracle, p, M, K, Ns, opA):
    """One saved A, several right-hand sides: bit-identical to plain calls and the oracle."""
    import torch
    A = synth.mp_random(500 + p, M, K, p, -20, 20)
    A.sign[3, :] = 0
    plan = oz.Plan.create(p, K)
    Ad = dev_mp(A.transpose() if opA else A)
    ra = oz.Residues(plan, Ad, oz.SIDE_A, op=opA)
    for i, N in enumerate(Ns):
        B = synth.mp_random(600 + p + i, K, N, p, -20, 20)
        Bd = dev_mp(B)
        print(f"reuse A: p={p} M={M} K={K} N={N} opA={opA}", flush=True)
        C1 = oz.gemm_from_residues(plan, B=Bd, ra=ra, opA=opA)
        C2 = oz.gemm(plan, Ad, Bd, opA, 0)
        torch.cuda.synchronize()
        assert _same(C1, C2), f"right-hand side {i}"
        _vs_oracle(C1, A, B, c_oracle)
    ra.destroy()


def test_reuse_right_operand_and_both(oz, c_oracle):
    """A saved B with several left-hand sides (op T), and both sides saved."""
    import torch
    p, K, N = 512, 150, 90
    B = synth.mp_random(701, K, N, p, -30, 30)
    plan = oz.Plan.create(p, K)
    Bd = dev_mp(B.transpose())
    rb = oz.Residues(plan, Bd, oz.SIDE_B, op=1)
    for i, M in enumerate((70, 129)):
        A = synth.mp_random(702 + i, M, K, p, -30, 30)
        Ad = dev_mp(A)
        print(f"reuse B: M={M}", flush=True)
        C1 = oz.gemm_from_residues(plan, A=Ad, rb=rb, opB=1)
        C2 = oz.gemm(plan, Ad, Bd, 0, 1)
        torch.cuda.synchronize()
        assert _same(C1, C2)
        _vs_oracle(C1, A, B, c_oracle)
        ra = oz.Residues(plan, Ad, oz.SIDE_A)
        C3 = oz.gemm_from_residues(plan, ra=ra, rb=rb)
        torch.cuda.synchronize()
        assert _same(C3, C2)
        ra.destroy()
    rb.destroy()


def test_reuse_errors(oz):
    p, M, K, N = 113, 40, 64, 30
    A = dev_mp(synth.mp_random(801, M, K, p, -4, 4))
    B = dev_mp(synth.mp_random(802, K, N, p, -4, 4))
    plan = oz.Plan.create(p, K)
    ra = oz.Residues(plan, A, oz.SIDE_A)
    rb = oz.Residues(plan, B, oz.SIDE_B)
    with pytest.raises(oz.Oz2hError) as ei:          # a handle of the wrong side
        oz.gemm_from_residues(plan, A=A, rb=ra)
    assert ei.value.code == oz.EINVAL
    other = oz.Plan.create(256, K)                   # another moduli set
    with pytest.raises(oz.Oz2hError) as ei:
        oz.gemm_from_residues(other, ra=ra, B=B)
    assert ei.value.code == oz.EINVAL
    rc = oz.lib().oz2h_gemm_from_residues(plan.handle, M, N, K, None, 0, A.cmat(), None, 0,
                                          B.cmat(), oz.empty_mp(M, N, p).mat(), None, 0, None)
    assert rc == oz.EINVAL                           # no handle at all
    with pytest.raises(oz.Oz2hError):
        oz.Residues(plan, A, 7)                      # bad side
    ra.destroy()
    rb.destroy()
