"""Host logic of bench.py: the stored counter profiles are reported only for
the kernel source and launch configuration they were taken on, and
`--gpus N` above 1 is refused."""
import subprocess
import sys
import types
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def _info(kernel, t2, t3, splits):
    return types.SimpleNamespace(kernel=[kernel, kernel], tile_t2=[t2, t2], tile_t3=[t3, t3],
                                 splits=[splits, splits])


def test_traffic_only_for_the_profiled_launch(monkeypatch):
    import hashlib
    src = "paper_2103_06393_amd/csrc/tv_dtg.hip"
    cur = hashlib.sha256((ROOT / src).read_bytes()).hexdigest()
    L = {"kernel": 2, "tile_t2": 128, "tile_t3": 4, "splits": 16}
    table = {("w", "fp32", "adjoint"): {"bytes": 123, "source": src, "sha256": cur,
                                         "profile": "profiles/dtg_c5_fp32_pmc.md",
                                         "launch": L},
             ("w", "fp32", "forward"): {"bytes": 456, "source": src, "sha256": "0" * 64,
                                         "profile": "profiles/dtg_c5_fp32_pmc.md",
                                         "launch": L}}
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", table)
    ok = _info(L["kernel"], L["tile_t2"], L["tile_t3"], L["splits"])
    assert bench.measured_traffic("w", "fp32", "adjoint", ok) == 123
    other = _info(L["kernel"], L["tile_t2"], L["tile_t3"], L["splits"] * 2)
    assert bench.measured_traffic("w", "fp32", "adjoint", other) is None
    fused = _info(1, L["tile_t2"], L["tile_t3"], L["splits"])
    assert bench.measured_traffic("w", "fp32", "adjoint", fused) is None
    assert bench.measured_traffic("w", "bf16x3", "adjoint", ok) is None
    # a changed kernel source voids the figure
    assert bench.measured_traffic("w", "fp32", "forward", ok) is None


def test_profiles_named_by_the_entries_exist():
    for e in bench.MEASURED_TRAFFIC.values():
        assert (ROOT / e["profile"]).is_file(), e["profile"]
        assert (ROOT / e["source"]).is_file(), e["source"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
