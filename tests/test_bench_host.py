"""Host logic of bench.py: algorithmic bytes and the counter-summary lookup."""
import os

import bench


def test_alg_bytes_two_step_counts_both_steps():
    one = bench.bytes_per_shot_launch(20, 1000, 800)
    assert one == 16 * 1000 + 20 * 800
    assert bench.bytes_per_shot_launch(20 | bench.TWO_STEP, 1000, 800) == 2 * one


def test_alg_bytes_fused_residual():
    """The fused residual update adds r's read and write to the adjoint pass
    (12 B per physical point with p's read, where N p's write was 4 of the 8)
    and nothing to the forward pass."""
    R = bench.RUPD
    assert bench.bytes_per_shot_launch(72 | R, 1000, 800) == 16 * 1000 + 12 * 800
    assert bench.bytes_per_shot_launch(20 | R, 1000, 800) == bench.bytes_per_shot_launch(20, 1000, 800)


def test_committed_summary_has_the_dominant_kernel():
    """The committed counter summary lists the fused forward and adjoint
    variants of the main leg."""
    text = open(bench.TRAFFIC_FILE).read()
    rows = {line.split("|")[1].strip().split()[0] for line in text.splitlines() if line.startswith("| ")}
    assert {str(20 | bench.RUPD), str(72 | bench.RUPD)} <= rows


def test_measured_traffic_lookup(tmp_path):
    h = bench.kernel_source_hash()
    text = "\n".join([
        f"kernel-sources-sha256-16: {h}  (note)",
        "calibration: fetch 2.0 write 1.0",
        "shots-per-launch: 16",
        "| launch | variant | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |",
        "|---|---|---:|---:|---:|",
        "| 20 56x32 | CG_FUSE+GATHER | 10 | 100.0 | 50.0 |",
        "| 20 56x24 | CG_FUSE+GATHER | 10 | 90.0 | 50.0 |",
        "| 72 56x32 | INJ+NORMAL | 10 | 10.0 | 5.0 |",
        "| 20 1step | CG_FUSE+GATHER | 10 | 30.0 | 20.0 |",
    ])
    p = tmp_path / "t.md"
    p.write_text(text)
    T = bench.TWO_STEP
    assert bench.measured_traffic(20 | T | (2 << 16), 16.0, str(p)) == (2 * 100 + 50) * 1024
    assert bench.measured_traffic(20 | T | (3 << 16), 16.0, str(p)) == (2 * 90 + 50) * 1024
    assert bench.measured_traffic(72 | T | (2 << 16), 16.0, str(p)) == (2 * 10 + 5) * 1024
    assert bench.measured_traffic(20, 16.0, str(p)) == (2 * 30 + 20) * 1024              # one step
    assert bench.measured_traffic(20 | T | (4 << 16), 16.0, str(p)) is None             # 40-row tiles not measured
    assert bench.measured_traffic(20 | T | (2 << 16), 8.0, str(p)) is None               # other shots per launch
    assert bench.measured_traffic(130 | T | (2 << 16), 16.0, str(p)) is None             # not measured
    p.write_text(text.replace(h, "0" * 16))
    assert bench.measured_traffic(20 | T | (2 << 16), 16.0, str(p)) is None              # kernels changed
    assert bench.measured_traffic(20 | T, 16.0, str(tmp_path / "missing.md")) is None


def test_launch_label():
    T = bench.TWO_STEP
    assert bench.launch_label(520) == "1step"
    assert bench.launch_label(520 | T | (3 << 16)) == "56x24"
    assert bench.launch_label(520 | T | (2 << 16), ndim=3) == "2step"


def test_committed_summary_parses():
    v = bench.measured_traffic(20 | bench.RUPD | bench.TWO_STEP | (2 << 16), 16.0)
    assert v is None or v > 0
    assert os.path.exists(bench.TRAFFIC_FILE)


def test_dense_bytes_per_cell_of_batching_variants():
    """Dense-stream bytes per physical cell and step, whatever the
    steps-per-launch bit: CORR|INJ (the adjoint with the correlation) reads the
    stored segment, 4; SRC_POINT|STORE (the recompute) writes it, 4; the
    fused-residual adjoint 12.  The gradient image a correlation adds into is
    an accumulator, not a stream of the method: PENALTY adds nothing to its
    dense source's 4."""
    T = bench.TWO_STEP
    assert bench.bench_dense_bytes(520 | T) == bench.bench_dense_bytes(520) == 4
    assert bench.bench_dense_bytes(257) == 4
    assert bench.bench_dense_bytes(72 | bench.RUPD) == 12
    assert bench.bench_dense_bytes(2 | 128) == 4
    # a launch's algorithmic bytes split into the padded and the dense parts
    assert bench.bytes_per_shot_launch(520 | T, 1000, 800) == 2 * (16 * 1000 + 4 * 800)


def test_roofline_object():
    r = bench.roofline("k", 8e9, 1000.0, 6e9, 5000.0)
    assert r["achieved"] == 8000.0 and r["frac"] == 1.0 and r["hbm_frac_counted"] == 0.75
    assert r["peak_measured"] == 5000.0 and r["frac_of_measured"] == 1.6
    assert bench.roofline("k", 8e9, 1000.0, None, None)["hbm_frac_counted"] is None


def test_unet_roofline():
    """The network's own ceiling: at least the FLOPs at the bf16 peak and the
    bytes of the full-resolution layers at the HBM peak; linear in the batch."""
    import bench
    one = bench.unet_roofline_us(408, 808, 1)
    assert abs(bench.unet_roofline_us(408, 808, 8) - 8 * one) < 1e-6 * one
    assert one * 1e-6 >= bench.unet_flops(408, 808) / 2.5e15
    # c1b alone: 16 channels in and out at 2 bytes, 808 x 408 pixels, at 8 TB/s
    assert one >= (16 + 16) * 2 * 808 * 408 / 8e12 * 1e6
