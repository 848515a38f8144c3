"""Pins of the oracle's momentum schedule (Alg. alg:prox-outer and
alg:prox-inner, the extrapolation step of each; Sec. 2.3.3).

The convergence pins elsewhere (NNLS, BVLS) hold for any reasonable
extrapolation weight, so they cannot tell the Beck-Teboulle weight
(t_k - 1)/t_{k+1} from the printed (t_k - 1)/(t_k + 1) or from a sequence
shifted by one.  These tests fix the first iterates exactly, on two problems
whose iterations are linear scalar recursions that can be written out by hand:

* outer iteration: A = I on one voxel, p = 1, no regulariser (the clamp at 0
  never acts), step alpha1 = 1/2.  The gradient step gives
  c_{k+1} = xi_k / 2 + 1/2, so with c_0 = xi_0 = 0:
      c_1 = 1/2, c_2 = 3/4 (beta_0 = 0), c_3 = (7 + b_1)/8,
      c_4 = (15 + b_1 + b_2 (1 + b_1))/16.
* inner (dual) iteration: one column of three voxels z = (0, 1, 2) along
  depth, radius theta = 10 (never reached).  The two edge duals stay equal,
  u = (s, s); grad z = (1, 1), grad grad^T = [[2, -1], [-1, 2]] and the step
  1/mu = 1/3 give s_{j+1} = (2/3) eta_j + 1/3, and the prox output is
  x = z - grad^T u = (s, 1, 2 - s):
      s_1 = 1/3, s_2 = 5/9 (beta_0 = 0), s_3 = (19 + 4 b_1)/27,
      s_4 = (65 + 8 b_1 + 8 b_2 (1 + b_1))/81.

b_k is the extrapolation weight of step k.  The step sequence of FISTA
(Beck and Teboulle 2009) starts at t_0 = 1 and obeys t_{k+1}^2 - t_{k+1} =
t_k^2, so t_1 is the golden ratio; its first values are written below as
decimals (checked against that identity here, not computed by the oracle).
"""
import math

import numpy as np
import pytest

import oracle
import oracle.core as core

# Beck-Teboulle step sequence t_0 .. t_4
T_SEQ = (1.0, 1.6180339887498948482, 2.1935270853310539386, 2.7497913401204452113,
         3.2948796779470478661)
# (t_k - 1)/t_{k+1}, k = 0..3
BT = (0.0, 0.28175352512532081819, 0.43404278278030200061, 0.53106380540447952985)
# printed form (t_k - 1)/(t_k + 1): b_1 = (phi - 1)/(phi + 1) = sqrt(5) - 2
LIT = (0.0, 0.23606797749978969641, 0.37373319638130706254, 0.46663698894356106241)

# hand-derived iterates (decimals of the closed forms in the docstring)
OUTER_BT = (0.5, 0.75, 0.91021919064066510227, 0.98988058700057355029)
OUTER_LIT = (0.5, 0.75, 0.90450849718747371205, 0.98112672585471022741)
INNER_BT = (1 / 3, 5 / 9, 0.74544496668523271381, 0.88524339674164709182)
INNER_LIT = (1 / 3, 5 / 9, 0.73867673740737625132, 0.87141013468398653221)


def _outer_closed(b):
    return (0.5, 0.75, (7 + b[1]) / 8, (15 + b[1] + b[2] * (1 + b[1])) / 16)


def _inner_closed(b):
    return (1 / 3, 5 / 9, (19 + 4 * b[1]) / 27, (65 + 8 * b[1] + 8 * b[2] * (1 + b[1])) / 81)


def test_step_sequence_literals():
    """The written t_k satisfy the FISTA identity, t_1 is the golden ratio and
    the weights are the two stated forms of them."""
    assert T_SEQ[1] == pytest.approx((1 + math.sqrt(5)) / 2, abs=1e-15)
    for k in range(4):
        assert T_SEQ[k + 1] ** 2 - T_SEQ[k + 1] == pytest.approx(T_SEQ[k] ** 2, abs=1e-13)
        assert BT[k] == pytest.approx((T_SEQ[k] - 1) / T_SEQ[k + 1], abs=1e-15)
        assert LIT[k] == pytest.approx((T_SEQ[k] - 1) / (T_SEQ[k] + 1), abs=1e-15)
    assert LIT[1] == pytest.approx(math.sqrt(5) - 2, abs=1e-15)
    np.testing.assert_allclose(_outer_closed(BT), OUTER_BT, atol=1e-15)
    np.testing.assert_allclose(_outer_closed(LIT), OUTER_LIT, atol=1e-15)
    np.testing.assert_allclose(_inner_closed(BT), INNER_BT, atol=1e-15)
    np.testing.assert_allclose(_inner_closed(LIT), INNER_LIT, atol=1e-15)


def _outer_iterates(literal=False):
    shape = (1, 1, 1, 1)
    p = np.ones(shape)
    out = []
    for k1 in range(1, 5):
        c, it = oracle.fista(p, lambda v: v, lambda w: w, 0.5, 0.0, 0.0, k1, 3,
                             shape_c=shape, literal_momentum=literal)
        assert it == k1
        out.append(float(c.ravel()[0]))
    return out


def _inner_iterates(literal=False):
    z = np.array([0.0, 1.0, 2.0]).reshape(1, 1, 1, 3)
    out = []
    for k2 in range(1, 5):
        x = oracle.prox_tv(z, 10.0, k2, literal_momentum=literal)
        # the iterate structure x = (s, 1, 2 - s)
        assert x[0, 0, 0, 1] == pytest.approx(1.0, abs=1e-15)
        assert x[0, 0, 0, 0] + x[0, 0, 0, 2] == pytest.approx(2.0, abs=1e-15)
        out.append(float(x[0, 0, 0, 0]))
    return out


def test_outer_iterates_beck_teboulle():
    np.testing.assert_allclose(_outer_iterates(), OUTER_BT, rtol=0, atol=1e-14)


def test_outer_iterates_printed_form():
    np.testing.assert_allclose(_outer_iterates(literal=True), OUTER_LIT, rtol=0, atol=1e-14)


def test_inner_iterates_beck_teboulle():
    np.testing.assert_allclose(_inner_iterates(), INNER_BT, rtol=0, atol=1e-14)


def test_inner_iterates_printed_form():
    np.testing.assert_allclose(_inner_iterates(literal=True), INNER_LIT, rtol=0, atol=1e-14)


def _shifted(t, literal=False):
    """A plausible mistake: the weight taken one step late, (t_{k+1}-1)/t_{k+2}."""
    t1 = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
    t2 = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t1 * t1))
    return t1, (t1 - 1.0) / t2


def _printed_as_default(t, literal=False):
    """Another: the printed form used where Beck-Teboulle's is meant."""
    t1 = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
    return t1, (t - 1.0) / (t + 1.0)


def _no_sqrt_update(t, literal=False):
    """Another: t advanced by one each step (t_k = k + 1), weight (t_k - 1)/t_{k+1}."""
    return t + 1.0, (t - 1.0) / (t + 1.0)


@pytest.mark.parametrize("wrong", [_shifted, _printed_as_default, _no_sqrt_update])
def test_pins_catch_a_wrong_schedule(monkeypatch, wrong):
    """With a wrong schedule planted in the oracle, both pins fail."""
    monkeypatch.setattr(core, "fista_momentum", wrong)
    assert not np.allclose(_outer_iterates(), OUTER_BT, rtol=0, atol=1e-9)
    assert not np.allclose(_inner_iterates(), INNER_BT, rtol=0, atol=1e-9)
