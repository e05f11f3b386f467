"""Host bookkeeping of the batch calls, checked without a GPU.

The library's host code (fz_api.hip, compiled for the host only, with the
address sanitizer) runs against a stand-in HIP runtime (tests/hipstub) that
tracks every allocation and every node a stream capture records.  Each graph
launch re-checks its nodes, so a captured kernel or copy that references
memory freed or reallocated since its capture fails the run, as do frees
that match no allocation, launches of destroyed graphs and leaked buffers.
The driver replays compression and decompression batches of growing sizes
and chain counts, interleaved, with replays, re-captures, single calls and
the autotuner's twelve captured launch configurations."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STUB = os.path.join(ROOT, "tests", "hipstub")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    if not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("hipcc or g++ not available")
    out = tmp_path_factory.mktemp("hipstub")
    flags = ["--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC", "-Wno-unused-value", "-Wno-unused-result",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    srcs = {"api": os.path.join(ROOT, "paper_2509_20563_amd", "csrc", "fz_api.hip"),
            "stub": os.path.join(STUB, "hip_stub.cpp"), "drv": os.path.join(STUB, "batch_replay.cpp")}
    objs = []
    for name, src in srcs.items():
        obj = str(out / f"{name}.o")
        r = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(out / "batch_replay")
    r = subprocess.run(["g++", "-fsanitize=address", *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_batch_graphs_never_touch_freed_memory(replay):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    r = subprocess.run([replay], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 stub errors, 0 failed checks" in r.stdout
