"""Host-side logic that needs no GPU: the autotuner's plane classes and its
JSON cache, and the benchmark's byte model."""
import json
import math

import pytest


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    P.load()
    return P


def test_plane_key_classes(P):
    from paper_1308_6644_amd import tune
    spec = dict(N=1024, type=2, lam=633e-9, z=0.1, g=4e-6, tf="asm", band="limited", tol=1e-6)
    assert tune.plane_key(spec, 1 << 20) == "plane:t2:N1024:w7:asm:m20"
    # the point count enters as round(log2 M); the width from the tolerance
    assert tune.plane_key(spec, 1_400_000) == "plane:t2:N1024:w7:asm:m20"
    assert tune.plane_key(dict(spec, tol=1e-9, tf="fresnel", band="full", type=1), 3000) == \
        "plane:t1:N1024:w10:fresnel:m12"
    assert tune.plane_key(dict(spec, tol=1e-2), 1) == "plane:t2:N1024:w3:asm:m0"


def test_tune_cache_round_trip(tmp_path):
    from paper_1308_6644_amd import tune
    path = tmp_path / "sub" / "tune.json"
    c = tune.TuneCache(str(path))
    assert c.get("plane:x") is None
    c.put("plane:x", {"spread_chunk": 896, "interp_chunk": 0, "bin_range_points": 0, "ms": 1.5})
    c.save()
    assert json.loads(path.read_text())["plane:x"]["spread_chunk"] == 896
    c2 = tune.TuneCache(str(path))
    assert c2.get("plane:x")["ms"] == 1.5


def test_cache_path_from_environment(monkeypatch, tmp_path):
    from paper_1308_6644_amd import tune
    monkeypatch.setenv("NUASM_TUNE_CACHE", str(tmp_path / "c.json"))
    assert tune.cache_path() == str(tmp_path / "c.json")


def test_bench_byte_model():
    """The per-launch algorithmic bytes of the spreading and interpolation
    kernels and the whole-path models at the headline size."""
    import bench
    info = dict(N=1024, Np=2048, L=2064, M=1 << 20, tiles=65 * 65, kx_lo=-1024, kx_hi=1023)
    M, L = 1 << 20, 2064
    assert bench.stage_bytes("spread", info) == 16 * M + 8 * M + 8 * L * L
    assert bench.stage_bytes("interp", info) == 8 * L * L + 16 * M + 8 * M
    assert bench.stage_bytes("t1_cols", info) == 8 * L * 2048 + 8 * 2048 * 2048
    # whole-path model of the survey: 302.0 MB (type 1) and 243.3 MB (type 2)
    Np = 2048
    assert math.isclose((64 * M + 56 * Np * Np) / 1e6, 302.0, abs_tol=0.1)
    assert math.isclose((56 * M + 44 * Np * Np) / 1e6, 243.3, abs_tol=0.1)


def test_bench_counters_follow_the_kernel_sources(tmp_path, monkeypatch):
    """Counter figures are used only while the kernel's sources are the ones
    they were taken on; the roofline's bound follows the counters."""
    import json
    import bench
    sha = bench.sources_sha256("spread")
    assert sha != bench.sources_sha256("t1_cols")
    path = tmp_path / "counters.json"
    rec = {"sources_sha256": sha, "fetch_bytes": 60e6, "write_bytes": 35e6, "valu_insts": 18e6,
           "mfma_insts": 1e6}
    path.write_text(json.dumps({"kernels": {"spread": rec, "t1_cols": dict(rec, sources_sha256="0" * 64)}}))
    monkeypatch.setattr(bench, "COUNTERS", str(path))
    assert bench.counter_record("spread")["valu_insts"] == 18e6
    assert bench.counter_record("t1_cols") is None      # taken on other sources
    assert bench.counter_record("interp") is None       # never taken
    # 1 launch of 60 us per step: VALU issue 18e6 x 4 / (1024 x 2.4e9 x 60e-6) = 0.49
    stages = {"spread": {"ms": 0.06, "launches": 1, "bytes": 50e6},
              "t1_cols": {"ms": 0.05, "launches": 1, "bytes": 50e6}}
    roof, report = bench.roofline(stages, 1)
    assert roof["kernel"] == "spread" and roof["bound"] == "alu"
    assert abs(roof["frac"] - 18e6 * 4 / (1024 * 2.4e9 * 60e-6)) < 1e-9
    assert roof["traffic"] == 95e6
    assert abs(roof["hbm_algorithmic_frac"] - 50e6 / 60e-6 / 8e12) < 1e-9
    # without counters the HBM roofline of the algorithmic bytes stays
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.json"))
    roof, _ = bench.roofline(stages, 1)
    assert roof["bound"] == "hbm" and roof["traffic"] is None
