"""Pins of the oracle's counter-based generator and of its propagation-region table.

Philox4x64-10 is checked bit for bit against numpy's independent implementation
(numpy advances the 256-bit counter by one before it generates a block, so the
block for counter c is numpy's first output for counter c - 1).  The region
table is checked against the invariants of the asymmetric checkerboard
propagation (Sec. 3.1): 4 near regions of 7 candidates, 4 far regions of 11,
all candidates of the other colour so that a half-pass is order independent.
"""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st


def numpy_block(ctr, key):
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    prev = [(v >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(4)]
    bg = np.random.Philox(counter=np.array(prev, np.uint64), key=np.array(key, np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((12345, 2, 1, 0), (7, 0)),
    ((2**64 - 1, 5, 2, 0), (2**63 + 11, 0)),
    ((0, 0, 3, 0), (1, 2)),  # counter word 0 = 0: numpy's borrow crosses words
])
def test_philox_matches_numpy(oracle_mod, ctr, key):
    assert np.array_equal(oracle_mod.philox4x64_10(ctr, key), numpy_block(ctr, key))


@settings(max_examples=60, deadline=None)
@given(st.lists(st.integers(0, 2**64 - 1), min_size=4, max_size=4), st.integers(0, 2**64 - 1))
def test_philox_matches_numpy_random(oracle_mod, ctr, seed):
    key = (seed, 0)
    assert np.array_equal(oracle_mod.philox4x64_10(ctr, key), numpy_block(ctr, key))


@settings(max_examples=200, deadline=None)
@given(st.integers(0, 2**64 - 1))
def test_uniform_top24_bits_exact(oracle_mod, w):
    u = oracle_mod.u24(w)
    assert 0.0 <= u < 1.0
    assert u * 2**24 == w >> 40
    assert float(np.float32(u)) == u  # exact in single precision too


def test_acp_table_invariants(oracle_mod):
    dx, dy, reg = oracle_mod.acp_offsets()
    assert len(dx) == 72
    offs = set(zip(dx.tolist(), dy.tolist()))
    assert len(offs) == 72, "offsets must be distinct"
    assert (0, 0) not in offs
    # every candidate has the other colour: odd Manhattan distance
    assert np.all((np.abs(dx) + np.abs(dy)) % 2 == 1)
    counts = np.bincount(reg, minlength=8)
    assert counts.tolist() == [7, 7, 7, 7, 11, 11, 11, 11]
    # reach: 23 px along the axes, near regions within 7 px (Manhattan)
    assert np.max(np.abs(dx) + np.abs(dy)) == 23
    near = reg < 4
    assert np.max(np.abs(dx[near]) + np.abs(dy[near])) <= 7
    # directions: up regions look up (dy < 0), down regions dy > 0, left dx < 0, right dx > 0
    for r, (sx, sy) in enumerate([(0, -1), (0, 1), (-1, 0), (1, 0)] * 2):
        m = reg == r
        if sy:
            assert np.all(np.sign(dy[m]) == sy)
        else:
            assert np.all(np.sign(dx[m]) == sx)
    # the four directions are 90-degree rotations of one another
    for fam in (0, 4):
        up = sorted(zip(dx[reg == fam].tolist(), dy[reg == fam].tolist()))
        left = sorted(zip(dx[reg == fam + 2].tolist(), dy[reg == fam + 2].tolist()))
        assert sorted((uy, ux) for ux, uy in up) == left
    # far regions are axial strips at odd distances 3..23
    far_up = sorted(dy[reg == 4].tolist())
    assert far_up == list(range(-23, -2, 2)) and np.all(dx[reg == 4] == 0)
