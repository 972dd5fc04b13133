"""AddressSanitizer + UBSan runs on the CPU.

* The C oracle built with gcc -fsanitize=address,undefined runs the oracle's
  pin tests (worked examples, brute force, invariants, edge slices).
* libnw with its host-only units (argument checks, layouts, the server and
  batch schedulers, the export driver) built with the same sanitizers runs the
  C-ABI tests, which exercise every host-side rejection path.

Each run is a child Python process with the matching sanitizer runtime
preloaded; every sanitizer report is fatal, and the child checks that the
sanitized library is the one it loaded.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import os, sys
import pytest
rc = pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu"] + sys.argv[1:])
maps = open("/proc/self/maps").read()
missing = [w for w in os.environ["NW_SAN_EXPECT"].split(",") if w not in maps]
if missing:
    print("sanitized libraries not loaded:", missing)
    sys.exit(3)
sys.exit(int(rc))
"""


def _run(env_extra, targets):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", CHILD] + targets, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, out
    return r


def test_oracle_pins_under_asan_and_ubsan():
    import oracle
    lib = oracle.build_sanitized()
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan), asan
    _run({"LD_PRELOAD": asan, "NW_ORACLE_LIB": lib, "NW_SAN_EXPECT": "liboracle_san.so,libasan"},
         ["tests/test_oracle_pins.py", "tests/test_edges_oracle.py", "tests/test_index_map.py"])


def test_abi_host_code_under_asan_and_ubsan():
    from paper_2509_01654_amd import build as nwbuild
    try:
        lib = nwbuild.build_host_sanitized()
    except RuntimeError as e:
        if "run build() first" not in str(e):
            raise
        nwbuild.build(verbose=False)
        lib = nwbuild.build_host_sanitized()
    rt = nwbuild.asan_runtime()
    _run({"LD_PRELOAD": rt, "NW_LIBRARY": lib, "NW_SAN_EXPECT": "libnw_hostsan.so,libclang_rt.asan"},
         ["tests/test_abi.py"])
