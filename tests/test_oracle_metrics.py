"""Pins of the oracle's two error metrics, the pass/fail gate of every parity
test: planted errors of known size must be reported exactly.

The metrics follow the parity bar of the dose product (Listing 1's per-voxel
sum in FP32 against the FP64 definition): the maximum per-voxel relative
error, and, for signed inputs (the adjoint's seed), the maximum error scaled
componentwise by |A| |x|.  Every planted value below is a power of two or a
small dyadic number, so the expected result is exact in FP64 and each check
is an equality.  The cases are chosen so that the plausible slips fail one of
them: dividing by |y| instead of |y*|, a mean instead of the maximum, the
zero-reference rule inverted or dropped, a signed instead of an absolute
difference, a scale taken from |y*| instead of the given one, and non-finite
results slipping through.
"""
import math

import numpy as np
import pytest

import oracle

TOL = 1e-5


def test_rel_err_reports_a_planted_error_exactly():
    y_ref = np.array([4.0, 8.0, 0.5, 3.0])
    y = y_ref.copy()
    y[1] = 8.0 * (1.0 + 2.0 ** -16)  # relative error 2^-16 ~ 1.5e-5
    assert oracle.max_rel_err(y, y_ref) == 2.0 ** -16
    assert not oracle.max_rel_err(y, y_ref) <= TOL
    y[1] = 8.0 * (1.0 - 2.0 ** -17)  # 7.6e-6: passes
    assert oracle.max_rel_err(y, y_ref) == 2.0 ** -17
    assert oracle.max_rel_err(y, y_ref) <= TOL


def test_rel_err_divides_by_the_reference_not_the_result():
    # |y - y*| = 1: relative to y* = 1 it is 1, relative to y = 2 it would be 1/2
    assert oracle.max_rel_err([2.0, 5.0], [1.0, 5.0]) == 1.0
    # and the other way round: y = 1 against y* = 2 gives 1/2 (not 1)
    assert oracle.max_rel_err([1.0], [2.0]) == 0.5


def test_rel_err_is_the_maximum_not_a_mean():
    y_ref = np.full(1000, 1.0)
    y = y_ref.copy()
    y[700] = 1.0 + 2.0 ** -10  # one bad voxel among 1000 good ones
    assert oracle.max_rel_err(y, y_ref) == 2.0 ** -10
    y[3] = 1.0 - 2.0 ** -8  # a larger error elsewhere, below the reference
    assert oracle.max_rel_err(y, y_ref) == 2.0 ** -8


def test_rel_err_zero_reference_rule():
    # exact zeros where the reference is zero: no error from them
    assert oracle.max_rel_err([0.0, 2.0], [0.0, 2.0]) == 0.0
    assert oracle.max_rel_err([-0.0, 2.0], [0.0, 2.0]) == 0.0
    # any nonzero value there is an unbounded error, however small
    assert oracle.max_rel_err([2.0 ** -149, 2.0], [0.0, 2.0]) == math.inf
    assert oracle.max_rel_err([-1e-30, 2.0], [0.0, 2.0]) == math.inf
    # all-zero reference and result
    assert oracle.max_rel_err(np.zeros(5), np.zeros(5)) == 0.0
    assert oracle.max_rel_err([], []) == 0.0


def test_rel_err_signed_values_use_absolute_differences():
    # y below y* by 2^-12 relative, with a negative reference
    assert oracle.max_rel_err([-1.0 + 2.0 ** -12], [-1.0]) == 2.0 ** -12
    assert oracle.max_rel_err([1.0 - 2.0 ** -12], [1.0]) == 2.0 ** -12


def test_rel_err_non_finite_results_fail():
    assert oracle.max_rel_err([np.nan, 1.0], [1.0, 1.0]) == math.inf
    assert oracle.max_rel_err([1.0, np.inf], [1.0, 1.0]) == math.inf
    assert oracle.max_rel_err([np.nan, 1.0], [0.0, 1.0]) == math.inf
    assert not oracle.max_rel_err([1.0, -np.inf], [1.0, 1.0]) <= TOL


def test_rel_err_rejects_mismatched_sizes():
    with pytest.raises(ValueError):
        oracle.max_rel_err([1.0, 2.0], [1.0])


def test_scaled_err_hand_worked_signed_example():
    # a row of a signed product: terms +3, -2, +1/2 give y* = 3/2 and
    # |A||x| = 11/2; an error of 2^-10 in y is 2^-10 / (11/2) relative to the scale
    y_ref = np.array([1.5, -0.25, 0.0])
    scale = np.array([5.5, 0.75, 2.0])
    y = np.array([1.5 + 2.0 ** -10, -0.25, 0.0])
    assert oracle.max_scaled_err(y, y_ref, scale) == 2.0 ** -10 / 5.5
    # a result whose reference is 0 but whose scale is not (cancellation) is
    # measured against the scale: 2^-20 / 2
    y[2] = -(2.0 ** -20)
    assert oracle.max_scaled_err(y, y_ref, scale) == 2.0 ** -10 / 5.5
    y[0] = 1.5
    assert oracle.max_scaled_err(y, y_ref, scale) == 2.0 ** -21


def test_scaled_err_uses_the_given_scale_not_the_reference():
    # reference -0.25 with scale 0.75: error 2^-8 gives 2^-8 / 0.75, not / 0.25
    got = oracle.max_scaled_err([-0.25 + 2.0 ** -8], [-0.25], [0.75])
    assert got == 2.0 ** -8 / 0.75
    assert got != 2.0 ** -8 / 0.25


def test_scaled_err_is_the_maximum_and_absolute():
    y_ref = np.zeros(100)
    scale = np.ones(100)
    y = np.zeros(100)
    y[10] = -(2.0 ** -9)  # negative deviation
    y[50] = 2.0 ** -12
    assert oracle.max_scaled_err(y, y_ref, scale) == 2.0 ** -9


def test_scaled_err_zero_scale_rule_and_non_finite():
    assert oracle.max_scaled_err([0.0, 1.0], [0.0, 1.0], [0.0, 1.0]) == 0.0
    assert oracle.max_scaled_err([-0.0, 1.0], [0.0, 1.0], [0.0, 1.0]) == 0.0
    assert oracle.max_scaled_err([2.0 ** -140, 1.0], [0.0, 1.0], [0.0, 1.0]) == math.inf
    assert oracle.max_scaled_err([np.nan, 1.0], [1.0, 1.0], [1.0, 1.0]) == math.inf
    assert oracle.max_scaled_err([1.0, np.inf], [1.0, 1.0], [1.0, 1.0]) == math.inf
    assert oracle.max_scaled_err(np.zeros(3), np.zeros(3), np.zeros(3)) == 0.0
    with pytest.raises(ValueError):
        oracle.max_scaled_err([1.0], [1.0], [1.0, 2.0])


CHECKS = [
    test_rel_err_reports_a_planted_error_exactly,
    test_rel_err_divides_by_the_reference_not_the_result,
    test_rel_err_is_the_maximum_not_a_mean,
    test_rel_err_zero_reference_rule,
    test_rel_err_signed_values_use_absolute_differences,
    test_rel_err_non_finite_results_fail,
    test_scaled_err_hand_worked_signed_example,
    test_scaled_err_uses_the_given_scale_not_the_reference,
    test_scaled_err_is_the_maximum_and_absolute,
    test_scaled_err_zero_scale_rule_and_non_finite,
]
