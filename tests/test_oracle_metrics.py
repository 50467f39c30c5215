"""Pins for the oracle's metrics and for its per-mode drop threshold.

* PSNR (Section 4): the textbook value of 8-bit data, 20 log10(255) = 48.1308... dB at a
  mean squared error of 1, with the peak taken from the approximation (not from the data).
* Principal angles between left interface subspaces (Definition 2) against scipy's
  subspace_angles on the materialised interfaces, including angles near 1e-10.
* Drop threshold of bfloat16 streams (Algorithm 3, step 5): on a tensor rounded to bf16
  the oracle's relative error (against the unrounded tensor) is within 1% of the float64
  run's, and the former threshold 3e-3 is shown to miss that bar.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import metrics, ttrbki
from tests.gpu_util import round_bf16


def test_psnr_textbook_8bit():
    # Xhat = 255 u o v o w with max |entry| exactly 255; X = Xhat + E with E = +-1 (MSE 1).
    rng = np.random.default_rng(0)
    u = rng.uniform(-1, 1, 6); u[2] = 1.0
    v = rng.uniform(-1, 1, 7); v[0] = -1.0
    w = rng.uniform(-1, 1, 5); w[4] = 1.0
    cores = [(255.0 * u).reshape(1, 6, 1), v.reshape(1, 7, 1), w.reshape(1, 5, 1)]
    Xhat = metrics.tt_full(cores)
    assert np.max(np.abs(Xhat)) == 255.0
    E = np.where(rng.random(Xhat.shape) < 0.5, -1.0, 1.0)
    E[2, 0, 4] = -1.0  # the peak entry 255 * 1 * -1 * 1 = -255 moves away from zero: |X| = 256 there
    X = Xhat + E
    assert np.max(np.abs(X)) == 256.0
    assert abs(metrics.psnr(X, cores) - 48.13080360867910) <= 1e-12
    # invariant under a common scale of data and approximation
    c2 = [cores[0] * 3.0, cores[1], cores[2]]
    assert abs(metrics.psnr(3.0 * X, c2) - 48.13080360867910) <= 1e-12


def _interface(cores, k):
    cur = cores[0].reshape(cores[0].shape[1], -1)
    for c in cores[1:k]:
        cur = (cur @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    return cur


@pytest.mark.parametrize("delta", [1e-1, 1e-4, 1e-10])
def test_interface_sines_against_scipy(delta):
    rng = np.random.default_rng(4)
    X = rng.standard_normal((5, 6, 4, 7))
    ranks = [3, 4, 3]
    a = ttrbki.tt_svd(X, ranks)
    b = ttrbki.tt_svd(X + delta * rng.standard_normal(X.shape), ranks)
    got = metrics.interface_sines(a, b)
    for k in range(1, 4):
        ua, ub = _interface(a, k), _interface(b, k)
        want = math.sin(float(np.max(scipy.linalg.subspace_angles(ua, ub))))
        assert abs(got[k - 1] - want) <= 1e-13 + 1e-7 * want, (k, got[k - 1], want)
    if delta == 1e-10:
        assert 1e-12 < max(got) < 1e-8


def test_interface_sines_gauge_invariant_and_orthogonal():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((4, 5, 6))
    cores = ttrbki.tt_svd(X, [3, 4])
    Rm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    g = [cores[0] @ Rm, np.einsum("ab,bic->aic", Rm.T, cores[1]), cores[2]]
    assert max(metrics.interface_sines(cores, g)) <= 1e-14
    # two mutually orthogonal one-dimensional interfaces: the sine is exactly one
    e0 = np.zeros((1, 4, 1)); e0[0, 0, 0] = 1.0
    e1 = np.zeros((1, 4, 1)); e1[0, 1, 0] = 1.0
    last = np.ones((1, 3, 1))
    assert metrics.interface_sines([e0, last], [e1, last]) == [1.0]


def test_bf16_rounded_input_matches_float64_error():
    w = synth.scaled_down(synth.workload("tt48x5"), (24, 24, 24, 24, 24))
    X = synth.build_host(w)
    Xb = round_bf16(X)
    args = (w.target_ranks(), w.q, w.p)
    e64 = metrics.rel_error(X, ttrbki.tt_rbki(X, *args, seed=0, precision="f64"))
    cores, modes = ttrbki.tt_rbki(Xb, *args, seed=0, precision="bf16", diagnostics=True)
    eb = metrics.rel_error(X, cores)
    assert [m.tau for m in modes] == [1e-5] * 4
    assert abs(eb - e64) <= 1e-2 * e64, (eb, e64)
    # the former bf16 threshold drops Krylov directions of the float32-carry modes
    e_old = metrics.rel_error(X, ttrbki.tt_rbki(Xb, *args, seed=0, tau=3e-3))
    assert abs(e_old - e64) > 1e-2 * e64, (e_old, e64)


def test_stream_precisions_follow_the_carry():
    modes = ttrbki.plan_modes([8] * 10, [16] * 9, q=2, p=8)
    assert ttrbki.stream_precisions("bf16", modes)[:3] == ["bf16", "bf16", "f32"]
    assert set(ttrbki.stream_precisions("f64", modes)) == {"f64"}
