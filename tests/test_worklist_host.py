"""Work lists of the pair sweeps, checked on the host (no GPU).

Compiles tests/host/worklist_check.cpp, which includes the library's C-ABI
translation unit and so builds the lists with the library's own builder,
links it against the built libcolatus.so for the kernel launchers it never
calls, and runs it: for single boxes from 1 to 2^16 particles, random ragged
batches and a 256-box ensemble it checks that the symmetric lists (grouped
and single-item) meet every unordered pair of parts once and write every
(particle, slot) their readers add exactly once, that the ordered lists
tile every box's sources, and that the allocation-free call's list
(generated on the device; here by the same functions, compiled for the
host) passes the same checks for N up to its limit and matches the
builder's grouped list item for item.
"""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1208_3444_amd")


def test_worklists_meet_every_pair_and_write_every_slot_once(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    assert os.path.exists(os.path.join(LIBDIR, "libcolatus.so")), "build the library first"
    exe = str(tmp_path / "worklist_check")
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I",
           os.path.join(ROOT, "include"), "-I", os.path.join(LIBDIR, "csrc"),
           os.path.join(ROOT, "tests", "host", "worklist_check.cpp"),
           os.path.join(ROOT, "tests", "host", "noalloc_list.cpp"), "-L", LIBDIR, "-lcolatus",
           "-Wl,-rpath," + LIBDIR, "-L", rocm_lib, "-lrocprofiler-sdk-roctx",
           "-Wl,-rpath," + rocm_lib, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0 and "all ok" in r.stdout, r.stdout[-4000:] + r.stderr[-2000:]
