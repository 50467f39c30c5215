"""CPU-side tests of the C ABI: the library loads, exports every declared entry
point, and the host-only planner validates, clamps and classifies exactly as the
step list (rank clamping and mode kinds of Algorithm 3 as read here) says."""
import ctypes
import os
import re

import pytest
import torch

import paper_2308_01480_amd as ttr
from oracle import ttrbki

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "ttrbki.h")).read()
    return sorted(set(re.findall(r"\b(ttr_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ttr.library_path())
    names = _declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    assert set(_declared_symbols()) <= set(ttr._SIGNATURES)


@pytest.mark.parametrize("name", ["tt20x4", "tt48x5", "odeco256x4", "tt8x10", "tt24x6"])
def test_plan_matches_step_list(name):
    import synth
    w = synth.workload(name)
    pl = ttr.plan(w.dims, w.ranks, w.q, w.p, torch.float32)
    modes = ttrbki.plan_modes(w.dims, w.target_ranks(), w.q, w.p)
    assert pl.kinds == [m.kind for m in modes]
    assert pl.ranks_list == [1] + [m.r for m in modes] + [1]
    for i, m in enumerate(modes):
        assert (pl.m[i], pl.n[i], pl.s[i], pl.w[i]) == (m.m, m.n, m.s, m.w)
    assert pl.workspace_bytes > 0
    assert pl.carry_dtype == ttr.TTR_F32


def test_plan_kinds_of_benchmark_shapes():
    pl = ttr.plan([48] * 5, 20, 3, 10, torch.float64)
    assert pl.kinds == ["saturated", "regular", "regular", "saturated"]
    assert list(pl.two_pass)[:4] == [0, 1, 1, 0]
    pl = ttr.plan([256] * 4, 32, 4, 8, torch.float32)
    assert pl.kinds == ["regular", "regular", "regular"]
    assert list(pl.two_pass)[:3] == [0, 1, 1]
    pl = ttr.plan([8] * 10, 16, 2, 8, torch.bfloat16)
    assert pl.ranks_list == [1, 8, 16, 16, 16, 16, 16, 16, 16, 8, 1]
    assert pl.kinds[0] == "identity" and pl.kinds[1] == "saturated"


def test_default_tau_by_dtype():
    # per mode from the data it streams: float64 1e-10, float32 and bfloat16 1e-5 (both
    # accumulate in float32); the plan reports the first mode's
    assert ttr.plan([10, 10, 10], 3, 1, 1, torch.float64).tau == 1e-10
    assert ttr.plan([10, 10, 10], 3, 1, 1, torch.float32).tau == 1e-5
    assert ttr.plan([10, 10, 10], 3, 1, 1, torch.bfloat16).tau == 1e-5
    assert ttr.plan([10, 10, 10], 3, 1, 1, torch.float64, tau=1e-7).tau == 1e-7


@pytest.mark.parametrize("dims,ranks,q,p", [
    ([10], [3], 1, 1),            # d < 2
    ([10, 0, 3], [2, 2], 1, 1),   # zero dim
    ([10, 5, 3], [2, 0], 1, 1),   # zero rank
    ([10, 5, 3], [2, 2], -1, 1),  # q < 0
    ([10, 5, 3], [2, 2], 1, -2),  # p < 0
])
def test_plan_rejects_bad_arguments(dims, ranks, q, p):
    with pytest.raises(ttr.TTRError, match="invalid argument"):
        ttr.plan(dims, ranks, q, p)


def test_plan_rejects_overflow_and_unsupported():
    with pytest.raises(ttr.TTRError, match="invalid argument"):
        ttr.plan([2 ** 32, 2 ** 32, 2 ** 32], [2, 2], 1, 1)
    with pytest.raises(ttr.TTRError, match="unsupported"):
        ttr.plan([200, 200, 200], [100, 100], 1, 1)


def test_rbki_argument_errors_enqueue_nothing():
    lib = ttr._load()
    dims = ttr._i64([4, 5, 6])
    rk = ttr._i64([2, 2])
    # null tensor pointer: rejected before any device work
    rc = lib.ttr_rbki(None, 0, 3, dims, rk, 1, 1, 0, None, None, None, 0, None)
    assert rc == -1
    assert b"null" in lib.ttr_last_error_detail()
    assert lib.ttr_strerror(-2) == b"workspace too small"


def test_gram_first_planning():
    # the 256^4 run parameters: the 256-row first mode takes the Gram form, the 8192-row
    # modes stream; forcing each form
    pl = ttr.plan([256] * 4, 32, 4, 8, torch.bfloat16)
    assert [pl.gram_first[k] for k in range(3)] == [1, 0, 0]
    pl = ttr.plan([256] * 4, 32, 4, 8, torch.bfloat16, krylov="streamed")
    assert [pl.gram_first[k] for k in range(3)] == [0, 0, 0]
    pl = ttr.plan([48] * 5, 20, 3, 10, torch.float32, krylov="gram")
    assert [pl.gram_first[k] for k in range(4)] == [0, 0, 0, 0]  # 960-row regular modes: too tall


def test_check_and_eigen_argument_errors():
    lib = ttr._load()
    # NULL names the allocation-free scratch of the current device: without a GPU (or
    # before any allocation-free call) there is none to read
    assert lib.ttr_check(None, None) in (-1, -3)
    assert lib.ttr_strerror(-4) == b"non-finite values"
    assert lib.ttr_sym_eig_workspace(128) >= 1 and lib.ttr_sym_eig_workspace(257) == 0
    assert lib.ttr_sym_eig_workspace(200) >= 200 * 256 * 8
    # n > 256 and missing scratch for n > 128 are refused before any device work
    assert lib.ttr_sym_eig(ctypes.c_void_p(8), 257, ctypes.c_void_p(8), ctypes.c_void_p(8), None, 0, None) == -1
    assert lib.ttr_sym_eig(ctypes.c_void_p(8), 200, ctypes.c_void_p(8), ctypes.c_void_p(8), None, 0, None) == -2


def test_workspace_starts_with_status_word():
    # the non-finite flag read by ttr_check sits in the first 256 bytes of both workspaces
    pl = ttr.plan([20, 20, 20, 20], 5, 2, 5, torch.float64)
    assert pl.workspace_bytes >= 256 and pl.grad_workspace_bytes > pl.workspace_bytes


def test_block_workspace_sizes():
    lib = ttr._load()
    assert lib.ttr_block_workspace(100, 1000, 10, 0) > 0
    assert lib.ttr_block_workspace(0, 1000, 10, 0) == 0
    assert lib.ttr_block_workspace(100, 1000, 65, 0) == 0


@pytest.mark.parametrize("m,n,s", [(960, 3000, 30), (960, 2304, 30), (1024, 1000, 32), (896, 5000, 16), (600, 777, 17),
                                   (960, 110592, 30)])
def test_block_workspace_holds_fused_register_variant_partials(m, n, s):
    """float32 unfoldings with 512 < m <= 1024 rows take the fused kernel that keeps Z in
    registers (S = 32, or S = 16 up to 896 rows): 16-column tiles, at most 256
    work-groups, m_pad x S float32 partials each.
    The block workspace (n x S stream buffer, partials, m_pad x S copy of Z) must hold
    them; the launch refuses to run otherwise."""
    lib = ttr._load()
    S = (s + 15) // 16 * 16
    m_pad = (m + 15) // 16 * 16
    groups = min((n + 15) // 16, 256)
    al = lambda v: (v + 255) // 256 * 256
    need = al(n * S * 4) + al(groups * m_pad * S * 4) + al(m_pad * S * 4)
    assert lib.ttr_block_workspace(m, n, s, 1) >= need


def test_no_cpu_fallback_for_host_tensors():
    # every compute entry takes device tensors only; a host tensor is an error, never a
    # silent CPU computation
    x = torch.zeros(4, 5, 6, dtype=torch.float64)
    with pytest.raises(ttr.TTRError, match="GPU tensor"):
        ttr.tt_rbki(x, [2, 2], 1, 1)
    with pytest.raises(ttr.TTRError, match="GPU tensor"):
        ttr.loss_grad(x, [2, 2], 1, 1)
    a = torch.zeros(8, 16, dtype=torch.float32)
    for call in (lambda: ttr.gram(a), lambda: ttr.carry(a, torch.zeros(8, 2, dtype=torch.float64)),
                 lambda: ttr.krylov(a, torch.zeros(8, 2, dtype=torch.float32))):
        with pytest.raises(ttr.TTRError, match="GPU tensor"):
            call()


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(ttr, "_lib", None)
    monkeypatch.setattr(ttr, "_LIB_PATH", str(tmp_path / "libttrbki.so"))
    with pytest.raises(ttr.TTRError, match="missing"):
        ttr.plan([4, 5, 6], [2, 2], 1, 1)
