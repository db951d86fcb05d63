"""Host-side checks of the C ABI (no GPU): symbols, argument errors, the planner."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_1209_4408_amd as gol

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(gol_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gol.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_string():
    assert "gfx950" in gol.version()
    assert isinstance(gol.lib().gol_last_error(), bytes)


@pytest.mark.parametrize("rows,cols,gens", [(0, 5, 1), (5, 0, 1), (3, 3, -1), (1 << 31, 4, 1)])
def test_step_rejects_bad_sizes(rows, cols, gens):
    buf = np.zeros(16, np.uint8)
    rc = gol.lib().gol_step(buf.ctypes.data, rows, cols, gens, buf.ctypes.data)
    assert rc == gol.GOL_EINVAL
    assert gol.lib().gol_last_error()


def test_step_rejects_null_and_partial_overlap():
    buf = np.zeros(64, np.uint8)
    assert gol.lib().gol_step(None, 4, 4, 1, buf.ctypes.data) == gol.GOL_EINVAL
    assert gol.lib().gol_step(buf.ctypes.data, 4, 4, 1, buf.ctypes.data + 3) == gol.GOL_EINVAL


def test_packed_rejects_bad_arguments():
    L = gol.lib()
    assert L.gol_step_packed(None, 4, 4, 1, 8, None) == gol.GOL_EINVAL
    assert L.gol_step_packed_ex(8, 4, 4, 1, 16, None, 3) == gol.GOL_EINVAL  # bad t_block
    assert L.gol_step_packed(8, 4, 70, 1, 16, None) == gol.GOL_EINVAL      # partial overlap
    assert L.gol_step_packed(8, 4, 4, -2, 64, None) == gol.GOL_EINVAL


def test_serve_create_rejects_bad_config():
    L = gol.lib()
    h = ctypes.c_void_p()
    bad = [gol.ServeConfig(1 << 20, -1, 0, 0, 0), gol.ServeConfig(0, 8, 0, 0, 0),
           gol.ServeConfig(1 << 20, 8, 0, 0, 3)]
    for cfg in bad:
        assert L.gol_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == gol.GOL_EINVAL
    assert L.gol_serve_poll(None, 1, None, None) == gol.GOL_EINVAL


def test_set_allocator_pairs():
    L = gol.lib()
    fn = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)(
        lambda n, s, c: None)
    assert L.gol_set_allocator(ctypes.cast(fn, ctypes.c_void_p), None, None) == gol.GOL_EINVAL
    assert L.gol_set_allocator(None, None, None) == gol.GOL_OK


# ---------------------------------------------------------------------------
# Planner
# ---------------------------------------------------------------------------
def check_plan(rows, cols, gens, T, band, chunk=False):
    out = gol.plan_tables(rows, cols, gens, T, band, chunk=chunk)
    segs, items, levels, late_begin, starts = out[:5]
    n = len(rows)
    K = [(g + T - 1) // T for g in gens]
    Kmax = max(K) if K else 0
    # every useful (row, dword) of every running board is written by exactly one lane
    cover = {b: np.zeros((rows[b], 2 * ((cols[b] + 63) // 64)), np.int32) for b in range(n)
             if K[b] > 0}
    for i, it in enumerate(items):
        late = i >= late_begin
        lanes = 0
        ss = segs[it["seg_begin"]: it["seg_begin"] + it["nseg"]]
        assert it["nseg"] >= 1
        mk = 0
        for s in ss:
            assert s["lane0"] == lanes, "segments are packed left to right"
            lanes += int(s["nlanes"])
            assert s["nlanes"] >= 3 and s["h"] >= 1 and s["h"] <= it["h"]
            b = int(s["board"])
            mk = max(mk, K[b])
            # a board of the late group ends at the last level, one of the early starts at 0
            assert starts[b] == (Kmax - K[b] if late else 0), (b, late, starts[b])
            D = 2 * ((cols[b] + 63) // 64)
            useful = np.arange(s["p0"] + 1, s["p0"] + s["nlanes"] - 1)
            assert useful.min() >= 0 and useful.max() < D
            cover[b][s["r0"]: s["r0"] + s["h"], useful] += 1
            if it["flags"] & 1:
                assert cols[b] % 32 == 0
        assert lanes <= 64
        assert it["maxK"] == mk
    for b, c in cover.items():
        assert (c == 1).all(), f"board {b} not covered exactly once"
    # each group's waves sorted by pass count; level L launches a prefix of each:
    # early waves with maxK > L, late waves with maxK >= Kmax - L
    me, ml = items["maxK"][:late_begin], items["maxK"][late_begin:]
    assert (np.diff(me) <= 0).all() and (np.diff(ml) <= 0).all()
    assert len(levels) == Kmax
    for L, (ce, cl) in enumerate(levels):
        assert ce == int((me > L).sum())
        assert cl == int((ml >= Kmax - L).sum())
    return segs, items, levels


@pytest.mark.parametrize("T", [1, 4, 8, 16])
def test_plan_covers_mixed_boards(T):
    rng = np.random.default_rng(5)
    rows = [int(x) for x in rng.integers(1, 300, 40)] + [1, 2, 3, 16384]
    cols = [int(x) for x in rng.integers(1, 3000, 40)] + [1, 2, 33, 16384]
    gens = [int(x) for x in rng.integers(0, 50, 40)] + [5, 0, 7, 3]
    check_plan(rows, cols, gens, T, 64)


def test_plan_batched_mix_shape():
    import seeded_inputs
    specs = seeded_inputs.batch_specs(1209, n=512)
    rows = [s.rows for s in specs]
    cols = [s.cols for s in specs]
    gens = [s.generations for s in specs]
    segs, items, levels = check_plan(rows, cols, gens, 8, 64)
    lanes_used = sum(int(s["nlanes"]) for s in segs)
    assert lanes_used / (64 * len(items)) > 0.7  # narrow boards share waves
    # early and late groups keep every level busy: without them the last levels
    # would hold only the few longest boards
    per_level = levels.sum(axis=1)
    assert per_level.min() > 0.5 * per_level.mean(), per_level


@pytest.mark.parametrize("T", [1, 8, 16])
@pytest.mark.parametrize("band", [0, 20, 96])
def test_chunk_plan_covers_mixed_boards(T, band):
    """A served chunk's schedule (each board tiled on its own) meets the
    same invariants, and no wave mixes boards."""
    rng = np.random.default_rng(11)
    rows = [int(x) for x in rng.integers(1, 400, 40)] + [1, 2, 3, 8192]
    cols = [int(x) for x in rng.integers(1, 3000, 40)] + [1, 2, 33, 8192]
    gens = [int(x) for x in rng.integers(0, 60, 40)] + [5, 0, 7, 3]
    segs, items, levels = check_plan(rows, cols, gens, T, band, chunk=True)
    for it in items:
        ss = segs[it["seg_begin"]: it["seg_begin"] + it["nseg"]]
        assert len(set(int(b) for b in ss["board"])) == 1


def test_chunk_plan_packs_bands_of_narrow_boards():
    # a 600 x 100 board has 4-dword strips (6 lanes with halos): ten of its
    # bands share each wave
    segs, items, levels, lb, starts, band = gol.plan_tables([600], [100], [32], 16, 20,
                                                           chunk=True)
    assert band == 20
    assert len(segs) == 30 and len(items) == 3
    assert (items["nseg"] == 10).all()


def test_chunk_band_model():
    """Few resident boards get short bands (more waves to fill the SIMDs),
    many get tall ones (less halo recompute)."""
    one = gol.plan_tables([512], [512], [240], 16, 0, chunk=True)[5]
    import seeded_inputs
    specs = seeded_inputs.serve_specs(1209, n=2048, rate_per_s=1.0)
    many = gol.plan_tables([s.rows for s in specs], [s.cols for s in specs],
                           [min(s.generations, 240) for s in specs], 16, 0, chunk=True)[5]
    assert one < many, (one, many)
    assert one >= 16 and many <= 256


def test_chunk_plan_time_is_linear():
    """Assembling a chunk from per-board tiles costs time linear in the tiles:
    4096 boards of the served mix take well under the build_plan search."""
    import time
    import seeded_inputs
    specs = seeded_inputs.serve_specs(1209, n=4096, rate_per_s=1.0)
    args = ([s.rows for s in specs], [s.cols for s in specs],
            [min(s.generations, 240) for s in specs])
    t0 = time.perf_counter()
    segs = gol.plan_tables(*args, 16, 96, chunk=True)[0]
    dt = time.perf_counter() - t0
    assert len(segs) > 50000
    assert dt < 1.0, dt


def test_plan_rejects_bad_input():
    with pytest.raises(gol.GolError):
        gol.plan_tables([4], [4], [-1])
    with pytest.raises(gol.GolError):
        gol.plan_tables([4], [4], [3], t_block=3)


@pytest.mark.parametrize("cfg", [dict(t_block=5), dict(t_block=12, layout=2),   # cols % 32 != 0
                                 dict(t_block=4, layout=2), dict(t_block=16, prefetch=3),
                                 dict(t_block=8, prefetch=12), dict(layout=4),
                                 dict(band_rows=-2), dict(t_block=16, layout=2, prefetch=6)])
def test_pass_config_rejected_before_any_device_work(cfg):
    """gol_step_packed_cfg checks the launch configuration on the host; the
    device pointers are never touched (they are not even valid here)."""
    c = gol.PassConfig(**{k: cfg.get(k, 0) for k in ("t_block", "band_rows", "prefetch",
                                                     "layout")})
    fake = ctypes.c_void_p(0x1000)
    rc = gol.lib().gol_step_packed_cfg(fake, 64, 100, 5, fake, None, ctypes.byref(c))
    assert rc == -1, (cfg, gol.lib().gol_last_error())


def test_paired_layout_needs_a_board_below_2_gib():
    c = gol.PassConfig(16, 0, 9, 2)
    fake = ctypes.c_void_p(0x1000)
    rc = gol.lib().gol_step_packed_cfg(fake, 131072, 131072, 5, fake, None, ctypes.byref(c))
    assert rc == -1
    assert b"2 GiB" in gol.lib().gol_last_error()


@pytest.mark.parametrize("checks,G", [([3, 2], 5), ([6], 5), ([-1], 5), ([0, 5, 4], 5)])
def test_population_checks_rejected_before_any_device_work(checks, G):
    """Checks must be non-decreasing generation counts within 0..generations; the
    call fails on the host, never touching the (invalid) device pointers."""
    ch = np.asarray(checks, dtype=np.int64)
    fake = ctypes.c_void_p(0x1000)
    rc = gol.lib().gol_step_packed_population(fake, 64, 100, G, fake, None, None,
                                              ch.ctypes.data, len(ch), fake)
    assert rc == -1, gol.lib().gol_last_error()
    assert b"checks" in gol.lib().gol_last_error()


def test_population_null_arguments():
    fake = ctypes.c_void_p(0x1000)
    L = gol.lib()
    assert L.gol_step_packed_population(fake, 64, 100, 5, fake, None, None, None, 2, fake) == -1
    ch = np.asarray([1], dtype=np.int64)
    assert L.gol_step_packed_population(fake, 64, 100, 5, fake, None, None, ch.ctypes.data, 1,
                                        None) == -1
    assert L.gol_population(None, 64, 100, fake, None) == -1
    assert L.gol_population(fake, 64, 100, None, None) == -1
    assert L.gol_population(fake, 0, 100, fake, None) == -1


def test_bounded_board_rejects_the_paired_layout():
    c = gol.PassConfig(12, 0, 9, 2)
    fake = ctypes.c_void_p(0x1000)
    rc = gol.lib().gol_step_packed_bounded(fake, 64, 128, 5, fake, None, ctypes.byref(c))
    assert rc == -1
    assert b"band layout" in gol.lib().gol_last_error()


@pytest.mark.parametrize("t,cfg,needle", [
    (3, None, b"t must be"), (0, None, b"t must be"), (-1, None, b"generations"),
    (17, None, b"t must be"),
    (8, gol.PassConfig(12, 0, 0, 0), b"t_block"), (8, gol.PassConfig(0, 0, 0, 2), b"band layout"),
    (8, gol.PassConfig(0, -1, 0, 0), b"negative"), (8, gol.PassConfig(0, 0, 4, 0), b"prefetch"),
])
def test_strip_pass_rejects_bad_arguments(t, cfg, needle):
    """Rejected before any device work (the pointers are never dereferenced)."""
    fake = [ctypes.c_void_p(0x100000 * k) for k in range(1, 5)]
    L = gol.lib()
    rc = L.gol_strip_pass(fake[0], fake[1], fake[2], 64, 128, t, fake[3], None,
                          ctypes.byref(cfg) if cfg is not None else None)
    assert rc == -1
    assert needle in L.gol_last_error(), L.gol_last_error()


def test_strip_pass_rejects_null_and_overlap():
    L = gol.lib()
    a, b, c, d = (ctypes.c_void_p(0x1000000 * k) for k in range(1, 5))
    assert L.gol_strip_pass(None, b, c, 64, 128, 4, d, None, None) == -1
    assert L.gol_strip_pass(a, None, c, 64, 128, 4, d, None, None) == -1
    assert L.gol_strip_pass(a, b, None, 64, 128, 4, d, None, None) == -1
    assert L.gol_strip_pass(a, b, c, 64, 128, 4, None, None, None) == -1
    assert L.gol_strip_pass(a, b, c, 0, 128, 4, d, None, None) == -1
    # 64 rows x 2 words = 1 KiB strip; outputs that touch the strip or a halo
    for out in (0x1000000, 0x1000000 + 1016, 0x2000000 + 8, 0x3000000 - 1000):
        rc = L.gol_strip_pass(a, b, c, 64, 128, 4, ctypes.c_void_p(out), None, None)
        assert rc == -1 and b"overlaps" in L.gol_last_error(), hex(out)


def test_resident_layout_rejects_boards_beyond_its_lds_budget():
    """rows x ceil(cols / 32) x 8 bytes must fit in 64 KiB (two generations)."""
    fake = ctypes.c_void_p(0x1000)
    L = gol.lib()
    c = gol.PassConfig(0, 0, 0, gol.LAYOUT_RESIDENT)
    rc = L.gol_step_packed_cfg(fake, 257, 1024, 5, ctypes.c_void_p(0x100000), None, ctypes.byref(c))
    assert rc == -1 and b"resident" in L.gol_last_error()
    c = gol.PassConfig(0, 0, 0, gol.LAYOUT_RESIDENT)
    rc = L.gol_step_packed_bounded(fake, 64, 64, 5, ctypes.c_void_p(0x100000), None, ctypes.byref(c))
    assert rc == -1 and b"band layout" in L.gol_last_error()


def test_valu_probe_rejects_bad_kinds_before_any_device_work():
    import ctypes as C
    L = gol.lib()
    r = C.c_double()
    assert L.gol_debug_valu_rate(-1, None, C.byref(r)) == -1
    assert L.gol_debug_valu_rate(5, None, C.byref(r)) == -1
    assert L.gol_debug_valu_rate(0, None, None) == -1


def test_binding_rejects_bad_host_buffers():
    """The binding checks every host buffer the library writes before the call:
    a short, wrongly typed, non-contiguous or read-only array is a ValueError,
    never an out-of-bounds write."""
    b = np.zeros((5, 70), np.uint8)
    for bad in (np.zeros((5, 69), np.uint8), np.zeros((5, 70), np.int32),
                np.zeros((5, 140), np.uint8)[:, ::2]):
        with pytest.raises(ValueError):
            gol.step(b, 1, out=bad)
    ro = np.zeros((5, 70), np.uint8)
    ro.flags.writeable = False
    with pytest.raises(ValueError):
        gol.step(b, 1, out=ro)
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=4, host_executor=True) as srv:
        w = np.zeros((6, 2), np.uint64)
        t = srv.submit(w, 6, 100, 3)
        for bad in (np.zeros((6, 1), np.uint64), np.zeros((6, 2), np.uint32),
                    np.zeros((6, 4), np.uint64)[:, ::2], np.zeros(11, np.uint64)):
            with pytest.raises(ValueError):
                srv.wait(t, bad)
            with pytest.raises(ValueError):
                srv.poll(t, bad)
        out = np.zeros((6, 2), np.uint64)
        srv.wait(t, out)  # the ticket is still good after the rejected calls
        with pytest.raises(gol.GolError) as e:
            srv.poll(t, out)
        assert e.value.code == gol.GOL_ENOTFOUND
        with pytest.raises(ValueError):
            srv.submit(np.zeros((6, 2), np.float64), 6, 100, 1)
        with pytest.raises(ValueError):
            srv.submit(np.zeros((6, 1), np.uint64), 6, 100, 1)


def test_binding_rejects_host_or_wrongly_sized_tensors():
    """Device entry points take device tensors of exactly rows * W int64 words;
    anything else is refused before the library sees a pointer."""
    import torch
    cpu = torch.zeros((4, 2), dtype=torch.int64)
    with pytest.raises(ValueError):
        gol.step_packed(cpu, 4, 100, 1)
    with pytest.raises(ValueError):
        gol.population(cpu, 4, 100)
    with pytest.raises(ValueError):
        gol.strip_pass(cpu, cpu, cpu, 4, 100, 1)
    with pytest.raises(ValueError):
        gol.batch_run([gol.BatchBoard(cpu, cpu, 4, 100, 1)])
