"""Host-side checks of bench.py's contract (no GPU needed).

* more than one GPU is refused with a message before anything touches a
  device (this build measures one GPU);
* the JSON line is strict: non-finite values become null;
* the traffic record of a kernel is used only for the kernel instantiation
  and the sources it was measured on;
* every committed profile summary names the command that made it.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_strict_json():
    import bench
    res = {"a": float("nan"), "b": [1.0, float("inf")], "c": {"d": -float("inf"), "e": 2}}
    line = json.dumps(bench._finite(res), allow_nan=False)
    assert json.loads(line) == {"a": None, "b": [1.0, None], "c": {"d": None, "e": 2}}


def test_traffic_record_matches_kernel_and_sources(tmp_path):
    import bench
    from paper_2305_05362_amd.build import kernel_digest
    kernel = "k_radial<float, 16>"
    rec = {"kernel": kernel, "kernel_name": "ram::" + kernel,
           "source_digest": kernel_digest(kernel), "traffic_bytes_per_launch": 1.0}
    path = tmp_path / "t.md"
    path.write_text("# x\n\n```json\n" + json.dumps(rec) + "\n```\n")
    assert bench.load_traffic(str(path), kernel)["traffic_bytes_per_launch"] == 1.0
    # another instantiation, or sources changed since: not used
    assert bench.load_traffic(str(path), "k_radial<double, 8>") is None
    rec["source_digest"] = "0" * 16
    path.write_text("# x\n\n```json\n" + json.dumps(rec) + "\n```\n")
    assert bench.load_traffic(str(path), kernel) is None
    # the step kernel's digest covers other sources than the radial kernel's
    assert kernel_digest("k_step_sh<float, 5, 3, 2, 0, 4, 1>") != kernel_digest(kernel)


@pytest.mark.parametrize("name", sorted(os.listdir(os.path.join(ROOT, "profiles"))))
def test_profiles_name_their_command(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert "rocprofv3" in text and "bench.py" in text

