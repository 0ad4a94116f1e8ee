"""Host-side checks of the benchmark's algorithmic byte models (no GPU)."""
import importlib.util
import os

import pytest

_spec = importlib.util.spec_from_file_location(
    "bench_model", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


@pytest.mark.parametrize("N,nb", [(4096, 32), (1000, 16), (257, 8)])
def test_panel_bytes_sum_over_columns(N, nb):
    # 4 * 8 * (N - c) bytes per column c: over a whole factorization the
    # per-launch figure times the launches is 4 * 8 * N (N + 1) / 2, and the
    # figure for launches that cover the first K columns is the column sum
    adv = nb - 1
    launches = (N + adv - 1) // adv
    whole = bench.panel_bytes_per_launch(N, launches) * launches
    assert whole == pytest.approx(4 * 8 * N * (N + 1) / 2)
    assert bench.panel_bytes_per_launch(N, launches, adv=adv) * launches == pytest.approx(whole)
    for n in (1, launches // 2, launches - 1):
        K = n * adv
        direct = sum(4 * 8 * (N - c) for c in range(K))
        assert bench.panel_bytes_per_launch(N, n, adv=adv) * n == pytest.approx(direct)


def test_trailing_bytes_small_case():
    # N = 10, panels of width 4: trailing matrices of order 6 and 2; the
    # lower triangle is read and written (no mirror), L and W read once
    got = bench.trailing_bytes_per_launch(10, 4)
    tot = 0.0
    for n in (6, 2):
        tot += 16.0 * n * (n + 1) / 2 + 2 * 8.0 * n * 4
    assert got == pytest.approx(tot / 2)
    got32 = bench.trailing_bytes_per_launch(10, 4, elem=4.0)
    tot32 = sum(8.0 * n * (n + 1) / 2 + 2 * 8.0 * n * 4 for n in (6, 2))
    assert got32 == pytest.approx(tot32 / 2)


@pytest.mark.parametrize("N", [4096, 16384, 2049, 1000])
def test_slot_plan_widths(N):
    # the widths cover the matrix; above 2048 rows every panel is nb - 1
    # wide, then 15 down to 1024 rows and 31 below (the library's plan)
    ws = bench.slot_widths(N)
    assert sum(ws) >= N and sum(ws[:-1]) < N
    rows = N
    for w in ws:
        assert w == (31 if rows > 2048 or rows <= 1024 else 15)
        rows -= w


def test_trailing_bytes_plan_reduces_to_uniform_width():
    # without a tail region (N <= 1024 rows: every panel 31 wide) the plan's
    # average equals the uniform-width model
    got, cnt = bench.trailing_bytes_plan(1000)
    assert got == pytest.approx(bench.trailing_bytes_per_launch(1000, 31))
    assert cnt == (1000 - 1) // 31
