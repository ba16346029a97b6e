"""Seeded synthetic inputs for the Ozaki-II p-bit GEMM.

This module only draws random numbers and lays them out in the operand
format; it holds none of the method's arithmetic.  Both the oracle's tests
and the GPU path's tests/bench take their inputs from here.
"""
from .gen import (MPMatrix, splitmix64, splitmix64_at, mp_random, mp_block, mp_zeros,
                  operands_for, operand_blocks_for, mp_unit_uniform, grad_operands_for,
                  limbs_for, CONFIG_SEED_BASE)

__all__ = ["MPMatrix", "splitmix64", "splitmix64_at", "mp_random", "mp_block", "mp_zeros",
           "operands_for", "operand_blocks_for",
           "mp_unit_uniform", "grad_operands_for",
           "limbs_for", "CONFIG_SEED_BASE"]
