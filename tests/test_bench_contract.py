"""The benchmark's command-line contract, checked on the CPU: more than one
GPU is refused with a message before anything touches a GPU, and `traffic`
comes from a counter summary only while the kernel sources it was taken on
are the current ones."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    for args, env in ((["--gpus", "2"], {}), (["--gpus", "8", "--steps", "1"], {}),
                      ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                           capture_output=True, text=True, timeout=120,
                           env={**os.environ, **env})
        assert r.returncode == 2, (args, r.stderr)
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_traffic_is_reported_only_for_the_profiled_sources():
    """Every committed counter summary and kernel trace names the hash of the
    kernel sources it was taken on, and bench.py reports `traffic` from a
    summary exactly when that hash is the current one (otherwise null)."""
    h = bench.kernel_source_hash()
    assert re.fullmatch(r"[0-9a-f]{16}", h)
    prof = os.path.join(ROOT, "profiles")
    names = sorted(os.listdir(prof))
    assert names, "no profiles"
    for n in names:
        assert re.search(r"kernel_source_hash: [0-9a-f]{16}", open(os.path.join(prof, n)).read()), n
    for form in bench.PROFILE_FORMS:
        if form == "stream_copy":
            continue
        path = os.path.join(prof, f"spinsum_{form}.traffic.txt")
        assert os.path.exists(path), form
        taken = re.search(r"kernel_source_hash: ([0-9a-f]{16})", open(path).read()).group(1)
        t = bench.traffic_from_profile(form)
        if taken == h:
            assert t is not None and t > 0, form
        else:
            assert t is None, form
