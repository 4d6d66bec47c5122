"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle and the input generator are rebuilt with both (any report aborts),
and the oracle's pins and the generator's tests run against those builds
in a child process.  No GPU code is involved."""
import os
import subprocess
import sys

import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]
PINS = ["test_oracle_assign.py", "test_oracle_ccl.py", "test_oracle_converge.py",
        "test_oracle_lab.py", "test_oracle_net.py", "test_oracle_seed.py",
        "test_oracle_stray.py", "test_oracle_update.py", "test_oracle_variants.py",
        "test_oracle_threads.py", "test_synth.py"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    flags = [f for f in oracle.CFLAGS if f != "-O3"] + ["-O1"] + SAN
    olib, slib = tmp_path / "liboracle_san.so", tmp_path / "libsynth_san.so"
    subprocess.run(["gcc", *flags, *oracle.SOURCES, "-o", str(olib), "-lm"], check=True)
    subprocess.run(["gcc", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-O1", *SAN, synth.SOURCE, "-o", str(slib), "-lm"],
                   check=True)
    env = dict(os.environ, SLIC_ORACLE_LIB=str(olib), SLIC_SYNTH_LIB=str(slib),
               LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider", *[os.path.join(ROOT, "tests", p) for p in PINS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
