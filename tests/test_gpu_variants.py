"""GPU parity of the other sweep drivers against the oracle's tt_variant: TT-rSVD
(Algorithm 2), TT-rSI (Algorithm 4) and TT-rBKI as printed (Algorithm 3 with the row-space
Krylov matrix), each with the printed first-r-columns truncation (literal) and, for rSVD
and rSI, with Rayleigh-Ritz.  Same bars as the TT-RBKI parity (test_gpu_sweep.run_pair).

The printed truncation keeps the span of an r-column power block; the GPU orthonormalises
each block rank-revealingly (directions below tau ||Y|| dropped and completed), while the
oracle's unpivoted Householder QR keeps them, so the cases use noisy tensors whose r-column
blocks are far from rank deficient."""
import numpy as np
import pytest

import synth
from tests.test_gpu_sweep import run_pair

pytestmark = pytest.mark.gpu

VARIANTS = [("rsvd", False), ("rsvd", True), ("rsi", False), ("rsi", True), ("rbki", True)]


def _cases():
    w = synth.scaled_down(synth.workload("tt24x6"), (10, 10, 10, 10, 10, 10))
    yield "tt24x6_small", synth.build_host(w), w.target_ranks(), w.q, w.p
    rng = np.random.default_rng(3)
    yield "tall-two-pass", rng.standard_normal((30, 30, 700)), [25, 10], 2, 5
    w = synth.scaled_down(synth.workload("power45x5_snr5"), (16,) * 5, ranks=4)
    yield "power16x5_snr5", synth.build_host(w), w.target_ranks(), w.q, w.p


CASES = list(_cases())


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("method,literal", VARIANTS)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_variant_parity(case, method, literal, dt):
    name, X, ranks, q, p = CASES[case]
    run_pair(X, ranks, q, p, 0, dt, name, method=method, literal=literal)
