"""Host checks of the constants the width-4 64-node round relies on.

The round tests move A's legality with one IEEE class test of a per-move
float constant against the node's move mask (bit A = move A allowed), so
each constant must belong to exactly class bit A of the class-test mask:
0 signaling NaN, 1 quiet NaN, 2 negative infinity, 3 negative normal.  The
classification below is written from the IEEE 754 binary32 encoding, not
from any library, and the constants are read from the kernel header.
"""
import os
import re

import pytest

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_1705_02843_amd", "csrc", "bpida_board.h")


def ieee_class_bit(bits):
    """Index of the class-test mask bit for a binary32 value: 0 sNaN,
    1 qNaN, 2 -inf, 3 -normal, 4 -denormal, 5 -0, 6 +0, 7 +denormal,
    8 +normal, 9 +inf."""
    sign = bits >> 31
    exp = (bits >> 23) & 0xFF
    frac = bits & 0x7FFFFF
    if exp == 0xFF:
        if frac:
            return 1 if frac & 0x400000 else 0
        return 2 if sign else 9
    if exp == 0:
        if frac == 0:
            return 5 if sign else 6
        return 4 if sign else 7
    return 3 if sign else 8


def header_constants():
    text = open(HEADER).read()
    found = dict((int(a), int(b, 16)) for a, b in re.findall(r"k\.cls\[(\d)\]\s*=\s*opaque_s\((0x[0-9A-Fa-f]+)u\)", text))
    assert sorted(found) == [0, 1, 2, 3], found
    return found


def test_classifier_on_known_values():
    assert ieee_class_bit(0x3F800000) == 8      # 1.0
    assert ieee_class_bit(0x80000000) == 5      # -0.0
    assert ieee_class_bit(0x00000001) == 7      # smallest denormal
    assert ieee_class_bit(0x7F800000) == 9      # +inf
    assert ieee_class_bit(0xFFC00000) == 1      # a quiet NaN with the sign set


@pytest.mark.parametrize("move", [0, 1, 2, 3])
def test_move_constant_is_in_class_bit_of_its_move(move):
    assert ieee_class_bit(header_constants()[move]) == move


def test_class_test_reads_only_bits_0_to_3_of_a_move_mask():
    # the round leaves the next cells' legal moves above bit 3 of the mask;
    # a constant of class bit A < 4 makes the test depend on bit A alone
    for move, c in header_constants().items():
        cls = ieee_class_bit(c)
        for mask in range(1 << 10):
            assert bool(mask >> cls & 1) == bool(mask >> move & 1)
