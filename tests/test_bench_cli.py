"""bench.py's command line on the CPU: more than one GPU is refused with a
message (the benchmark measures one GPU), and the byte model the roofline divides
by matches the per-unit bytes stated for the kernels."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_roofline_byte_model():
    """Per line unknown: gathered value, chord, |beta| (beta family), load (beta
    family, FP64 sweeps only: the FP32 increment sweeps have no source), written
    value; tables: cell index and two cell offsets.  Per grid node: each line
    value read once, plus the grid traffic of the scatter mode; tables: slot
    index, record base, three offsets and the record weights."""
    sys.path.insert(0, ROOT)
    import bench
    assert [bench.line_bytes(*k)[0] for k in (("fp32", 0), ("fp32", 1), ("fp64", 0), ("fp64", 1))] == \
        [16, 12, 40, 24]
    assert [bench.line_bytes(*k)[1] for k in (("fp32", 0), ("fp64", 1))] == [12, 20]
    counts = dict(grid_unknowns=1000, line_unknowns_b=1000, lines_b=10, line_unknowns_g=800, lines_g=20)
    alg = [bench.scatter_bytes(p, f, counts)[0] for p, f in (("fp32", 0), ("fp32", 1), ("fp64", 0), ("fp64", 1))]
    assert alg == [4 * 1.02 + 4, 4 * 0.84 + 20, 8 * 1.02 + 8, 8 * 0.84 + 20]
    assert bench.scatter_bytes("fp64", 1, counts, march=True)[0] == 8 * 0.84 + 8
    assert [bench.scatter_bytes(p, 0, counts)[1] for p in ("fp32", "fp64")] == [26, 66]
    # direct transfer: source value, chord, |beta| and load (beta, FP64), written value; gamma: the
    # update traffic (FP64: old value + FP32 increment; FP32: FP64 state read and written);
    # tables: two bracket indices and four weights (FP64), or 10 packed bytes (FP32 sweeps)
    assert [bench.direct_line_bytes(*k) for k in (("fp32", 0), ("fp32", 1), ("fp64", 0), ("fp64", 1))] == \
        [(16, 10), (28, 10), (40, 40), (36, 40)]


def test_roofline_from_kernel_work():
    """The roofline divides the algorithmic bytes of the work the library
    counted per launch by the summed event time; the dominant class is the one
    with the largest total time."""
    sys.path.insert(0, ROOT)
    import bench
    counts = dict(grid_unknowns=1000, line_unknowns_b=1000, lines_b=10, line_unknowns_g=800, lines_g=20)
    z = (0.0, 0, 0)
    times = {"fp64": {"line_beta": (1.0, 2, 2000), "line_gamma": z, "scatter_beta": z, "scatter_gamma": z,
                      "norm": z},
             "fp32": {"line_beta": (2.0, 4, 4000), "line_gamma": z, "scatter_beta": (0.5, 4, 4000),
                      "scatter_gamma": z, "norm": z}}
    rf = bench.roofline(times, counts)
    assert rf["kernel"] == "k_line<float, 0, false>"
    assert abs(rf["achieved"] - 16 * 4000 / 2e-3 / 1e9) < 0.1
    assert rf["bytes_per_launch"] == 16 * 1000
    assert [c["cls"] for c in rf["classes"]] == ["line_beta", "line_beta", "scatter_beta"]


def test_roofline_of_the_direct_increments_on_the_grid_route():
    """Direct increments steering the grid route: the FP32 line classes are
    the direct line kernels (the gamma one adds to an FP32 sum, 4 B read and
    written), class scatter_beta is the block's gather onto the gamma-curves
    (grid value, curve value, cleared sum; bilinear stencil as tables) and
    scatter_gamma the FP32 increment scatter; the FP64 classes are unchanged."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.direct_line_bytes("fp32", 1, hybrid=True) == (20, 10)
    assert bench.hybrid_gather_bytes() == (12.0, 12.0)
    counts = dict(grid_unknowns=1000, line_unknowns_b=1000, lines_b=10, line_unknowns_g=800, lines_g=20)
    z = (0.0, 0, 0)
    times = {"fp64": {"line_beta": (0.5, 1, 1000), "line_gamma": z, "scatter_beta": z,
                      "scatter_gamma": (0.4, 1, 1000), "norm": z},
             "fp32": {"line_beta": (2.0, 4, 4000), "line_gamma": (1.5, 4, 3200), "scatter_beta": (0.2, 1, 800),
                      "scatter_gamma": (0.3, 1, 1000), "norm": z}}
    rf = bench.roofline(times, counts, hybrid=True)
    names = {(c["prec"], c["cls"]): c["kernel"] for c in rf["classes"]}
    assert names[("fp32", "line_beta")] == "k_line<float, 0, true>"
    assert names[("fp32", "line_gamma")] == "k_line<float, 1, true>"
    assert names[("fp32", "scatter_beta")] == "k_line_values<float>"
    assert names[("fp32", "scatter_gamma")] == "k_scatter<float, double, 2>"
    assert names[("fp64", "line_beta")] == "k_line<double, 0, false>"
    assert names[("fp64", "scatter_gamma")] == "k_scatter<double, double, 1>"
    row = {(c["prec"], c["cls"]): c for c in rf["classes"]}
    assert row[("fp32", "line_gamma")]["alg_bytes_per_unit"] == 20
    assert row[("fp32", "scatter_beta")]["alg_bytes_per_unit"] == 12
    assert rf["kernel"] == "k_line<float, 0, true>"


def test_measured_traffic_of_a_bucketed_class(tmp_path, monkeypatch):
    """A bucketed line class sums its kernels' rows (one dispatch per bucket
    shape) from a summary taken on the current kernel sources; other sources
    give None."""
    import hashlib
    sys.path.insert(0, ROOT)
    import bench
    h = hashlib.sha256()
    for f in ("adr_kernels.hip", "adr_kernels.h"):
        with open(os.path.join(ROOT, "paper_2411_11041_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    prof = tmp_path / "profiles"
    prof.mkdir()
    rows = ["| adr::k_line_b<float, 1, 4, 256, true> | 1 | 2 | 3.0e+06 |",
            "| adr::k_line_b<float, 1, 8, 64, true> | 1 | 2 | 1.5e+06 |",
            "| adr::k_line_b<float, 0, 4, 256, true> | 1 | 2 | 9.0e+06 |",
            "| adr::k_line_b<float, 1, 4, 256, false> | 1 | 2 | 7.0e+06 |",
            "| adr::k_line<float, 1, true> | 1 | 2 | 2.0e+06 |"]
    (prof / "x.md").write_text(f"Kernel source sha256[:16] = {h.hexdigest()[:16]}\n" + "\n".join(rows) + "\n")
    (prof / "old.md").write_text("Kernel source sha256[:16] = 0000000000000000\n" + "\n".join(rows) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the kernel sources are read from ROOT too: point them at the real tree
    real = os.path.join(ROOT, "paper_2411_11041_amd")
    os.symlink(real, tmp_path / "paper_2411_11041_amd")
    name = bench.kernel_name("fp32", "line_gamma", 1, direct=True)
    assert bench.measured_traffic(name, "x.md") == 4.5e6
    assert bench.measured_traffic("k_line<float, 1, true>", "x.md") == 2.0e6
    assert bench.measured_traffic(name, "old.md") is None
    assert bench.measured_traffic(name, "missing.md") is None
