"""The algorithmic-byte models behind bench.py's bandwidth figures, checked
against the per-cell counts they are built from (no GPU needed)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(spec)
spec.loader.exec_module(bench)

N = 128 * 128 * 32


def test_spmv_bytes_are_552_per_cell_plus_rhs_once_per_cycle():
    tot, launches = bench.algorithmic_bytes("spmv", 3, N, [15], "fp64")
    assert launches == 16
    assert tot == 15 * 552 * N + (552 + 24) * N
    tot2, launches2 = bench.algorithmic_bytes("spmv", 3, N, [30, 5], "fp64")
    assert launches2 == 37 and tot2 == 35 * 552 * N + 2 * (552 + 24) * N


def test_orth_bytes_count_each_basis_vector_once_per_pass():
    # CGS2, step j of a cycle: three passes over nv = j + 1 vectors plus w
    tot, launches = bench.algorithmic_bytes("orth", 3, N, [2], "fp64", orth="cgs2")
    per = 3 * 8 * N
    assert launches == 6
    assert tot == ((1 + 1) + (1 + 2) + (1 + 2)) * per + ((2 + 1) + (2 + 2) + (2 + 2)) * per
    # delayed CGS2, step j: dots over j vectors + uh + w, update over j
    # vectors + uh + w read and v_j, u written
    tot, launches = bench.algorithmic_bytes("orth", 3, N, [2], "fp64")
    assert launches == 4
    assert tot == ((0 + 2) + (0 + 4)) * per + ((1 + 2) + (1 + 4)) * per
    # two passes instead of three: a third fewer bytes over a 30-step cycle
    c2, _ = bench.algorithmic_bytes("orth", 3, N, [30], "fp64", orth="cgs2")
    d2, _ = bench.algorithmic_bytes("orth", 3, N, [30], "fp64")
    assert 0.6 < d2 / c2 < 0.7


def test_smoother_counts_only_the_multi_block_levels():
    levels = [N, N // 8, N // 64, N // 512, 128]
    tot, launches = bench.algorithmic_bytes("smooth", 3, N, [15], "fp64", levels=levels)
    # levels above the first one of at most 4096 cells: three half-sweeps each
    assert launches == 15 * 3 * 3
    assert tot == 15 * (44 + 41 + 40) * (N + N // 8 + N // 64)


def test_smoother_counts_the_extra_sweeps_of_a_longer_cycle():
    # V(2,2): one more red + black-pre pair before and one more black-pre +
    # red pair after the coarse correction on every multi-block level
    levels = [N, N // 8, N // 64, N // 512, 128]
    t1, l1 = bench.algorithmic_bytes("smooth", 3, N, [15], "fp64", levels=levels)
    t2, l2 = bench.algorithmic_bytes("smooth", 3, N, [15], "fp64", levels=levels, pre=2, post=2)
    assert l2 == 15 * 3 * 7 and l2 - l1 == 15 * 3 * 4
    assert t2 - t1 == 15 * 2 * (40 + 44) * (N + N // 8 + N // 64)


def test_ilu_bytes_match_the_colour_sweep_formulas():
    tot, launches = bench.algorithmic_bytes("ilu", 3, N, [15], "fp64")
    b, nh = 3, N // 2
    per = nh * 8 * ((b * b + 9 * b) + (7 * b * b + 5 * b) + (7 * b * b + 3 * b + 1)) + 2 * N * 8
    assert launches == 45 and tot == 15 * per
    # 764 B per cell and application at b = 3, as the kernel table states
    assert ((b * b + 9 * b) + (7 * b * b + 5 * b) + (7 * b * b + 3 * b + 1)) * 8 // 2 + 2 * 8 == 764


def test_network_flop_model():
    # 2 * 27 * C_in * C_out per output voxel of each level, plus the head
    v0 = N
    conv = sum(2 * 27 * ci * co * v0 // 8 ** lv for ci, co, lv in bench.NET_CONVS)
    assert bench.network_flop(128, 128, 32) == conv + 2 * 16 * v0
    assert abs(bench.network_flop(128, 128, 32) / 1e9 - 27.88) < 0.05
