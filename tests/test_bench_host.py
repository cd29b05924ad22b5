"""Host-side logic of bench.py (no GPU): the binding roofline follows the larger of the two
algorithmic floors, and the committed traffic figure is only reported for the sources it was
measured on."""
import os

import bench


def test_roofline_binds_hbm_at_nside_2048():
    # one FP32 map in and out at Nside 2048 (402,653,184 bytes) and its 48,266,767,192 pixel pairs
    r = bench.roofline_for("mixed_persistent_kernel", 3.0, 48266767192, 402653184)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["floor_us"] - 50.331648) < 1e-9
    assert abs(r["achieved"] - 402653184 / 3.0e-3 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-15
    other = r["other_roofline"]
    assert other["bound"] == "mfma" and abs(other["floor_us"] - 2 * 48266767192 / 2.5e15 * 1e6) < 1e-9
    assert r["traffic"] is None          # only for the profiled configuration


def test_roofline_binds_flops_when_pairs_dominate():
    r = bench.roofline_for("pair_accumulate_kernel", 100.0, 48266767192, 402653184)
    assert r["bound"] == "alu" and r["peak"] == 78.6


def test_traffic_note_matches_sources_or_is_ignored(tmp_path, monkeypatch):
    note = tmp_path / "note.md"
    note.write_text("source_sha256: `deadbeef`\nhbm_bytes_per_launch: `123`\n")
    monkeypatch.setattr(bench, "TRAFFIC_NOTE", str(note))
    assert bench.measured_traffic() is None
    note.write_text(f"source_sha256: `{bench.kernel_source_hash()}`\nhbm_bytes_per_launch: `123`\n")
    assert bench.measured_traffic() == 123.0
    monkeypatch.setattr(bench, "TRAFFIC_NOTE", os.path.join(str(tmp_path), "missing.md"))
    assert bench.measured_traffic() is None


def test_source_hash_follows_code_not_comments(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    src.write_text("int f(int a) {  // doubles\n  return 2 * a; /* twice */ }\n")
    h0 = bench.kernel_source_hash()
    src.write_text("// a header comment\nint f(int a) {\n  /* the value, twice\n   over */\n  return 2 * a;  }\n")
    assert bench.kernel_source_hash() == h0
    src.write_text("int f(int a) { return 3 * a; }\n")
    assert bench.kernel_source_hash() != h0


def test_paper_context_is_eq7():
    # Eq. 7 at theta_cut = 30 arcmin: 0.0232 s x 30 + 2.428 s = 3.124 s per Nside 2048 map
    import math
    c = bench.paper_context(30.0 / 60.0 * math.pi / 180.0, 48266767192, 400.0)
    assert abs(c["seconds_per_map"] - 3.124) < 1e-12
    assert abs(c["maps_per_s"] - 1.0 / 3.124) < 1e-12
    assert abs(c["ratio_maps_per_s_here"] - 400.0 * 3.124) < 1e-9


def test_check_pixels_cover_poles_and_belt_edges():
    # the batched leg's check pixels: the seeded uniform ones plus the first, middle and last pixel
    # of the polar rings and of the rings beside both belt edges (ring starts from the oracle's table)
    import numpy as np

    from oracle import geometry
    for nside in (1, 2, 4, 16, 256):
        pix = bench.check_pixels(nside, 300, 5)
        rt = geometry.ring_table(nside)
        npix = 12 * nside * nside
        assert pix.min() >= 0 and pix.max() < npix and np.all(np.diff(pix) > 0)
        N = nside
        for i in {1, 2, N - 1, N, N + 1, 3 * N - 1, 3 * N, 3 * N + 1, 4 * N - 2, 4 * N - 1}:
            if 1 <= i <= 4 * N - 1:
                s0, n = int(rt["start"][i - 1]), int(rt["n"][i - 1])
                assert {s0, s0 + n // 2, s0 + n - 1} <= set(pix.tolist()), (nside, i)
        assert len(pix) >= min(300, npix)
