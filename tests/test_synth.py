"""The input generator's block and torch forms equal its plain numpy form (CPU)."""
import numpy as np
import pytest

import synth


def test_block_equals_slice():
    M, N, K, p = 9, 7, 11, 130
    A, B = synth.operands_for(5, M, N, K, p, -16, 16)
    a, b = synth.operand_blocks_for(5, M, N, K, p, -16, 16, range(2, 6), range(3, 7))
    assert np.array_equal(a.sign, A.sign[2:6]) and np.array_equal(a.exp, A.exp[2:6])
    assert np.array_equal(a.limbs, A.limbs[2:6])
    assert np.array_equal(b.sign, B.sign[:, 3:7]) and np.array_equal(b.exp, B.exp[:, 3:7])
    assert np.array_equal(b.limbs, B.limbs[:, 3:7])


@pytest.mark.parametrize("p,lo,hi", [(2, -3, 3), (64, -32, 32), (113, -16, 16), (2048, -16, 16)])
def test_torch_generator_equals_numpy(p, lo, hi):
    torch = pytest.importorskip("torch")
    from synth.gen_torch import operands_for_torch
    M, N, K = 13, 6, 21
    A, B = synth.operands_for(77, M, N, K, p, lo, hi)
    (sa, ea, la), (sb, eb, lb) = operands_for_torch(77, M, N, K, p, lo, hi, device="cpu")
    assert np.array_equal(sa.numpy(), A.sign) and np.array_equal(ea.numpy(), A.exp)
    assert np.array_equal(la.numpy().view(np.uint64), A.limbs)
    assert np.array_equal(sb.numpy(), B.sign) and np.array_equal(eb.numpy(), B.exp)
    assert np.array_equal(lb.numpy().view(np.uint64), B.limbs)
