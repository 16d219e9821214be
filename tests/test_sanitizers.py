"""CPU sanitizer tier: the library's host code (factor.cpp, api.cpp), the CPU
replay of the GPU decompositions (tests/emu/chunk_emu.cpp) and the oracle
(oracle/bb_oracle.c), built with AddressSanitizer (leak checks included) and
UndefinedBehaviorSanitizer and driven by tests/san/san_main.cpp: factors of
every kind and size class (one-launch and long systems), their plans, every
argument and pivot error, the Cahn-Hilliard factor, and the replayed
decompositions against the oracle.  The device objects of the library are
linked unsanitised; no device call is made."""
import os
import subprocess

import pytest

from paper_2107_05395_amd import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2107_05395_amd", "csrc")
KOBJ = os.path.join(ROOT, "_build")
OUT = os.path.join(ROOT, "_build", "san")
# every device unit of the library, as the build lists them
DEVICE_UNITS = [s[:-len(".hip")] for s in _build.SOURCES if s.endswith(".hip")]
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]
HIP = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr)
    return res


@pytest.fixture(scope="module")
def san_binary():
    if not all(os.path.exists(os.path.join(KOBJ, u + ".o")) for u in DEVICE_UNITS):
        _build.build(verbose=False)
    os.makedirs(OUT, exist_ok=True)
    units = [("g++", os.path.join(CSRC, "api.cpp"), ["-std=c++17"] + HIP),
             ("g++", os.path.join(CSRC, "factor.cpp"), ["-std=c++17"] + HIP),
             ("g++", os.path.join(HERE, "emu", "chunk_emu.cpp"), ["-std=c++17"] + HIP),
             ("g++", os.path.join(HERE, "san", "san_main.cpp"), ["-std=c++17"] + HIP),
             ("gcc", os.path.join(ROOT, "oracle", "bb_oracle.c"),
              ["-std=c11", "-fopenmp", "-ffp-contract=off"])]
    objs = []
    for cc, src, flags in units:
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        _run([cc, *flags, *SAN, "-c", src, "-o", obj])
        objs.append(obj)
    exe = os.path.join(OUT, "san_run")
    _run(["g++", *SAN, "-fopenmp", "-o", exe, *objs,
          *(os.path.join(KOBJ, u + ".o") for u in DEVICE_UNITS),
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    return exe


def test_host_code_under_address_and_undefined_sanitizers(san_binary):
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([san_binary], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "sanitizer run ok" in res.stdout
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr
