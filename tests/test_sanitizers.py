"""The C code under sanitizers, on the CPU: the oracle (every entry point,
the analysis on four threads) under AddressSanitizer and
UndefinedBehaviorSanitizer, then ThreadSanitizer; the host side of libpaam
(validation, derivation and packing of a batch on up to 16 threads, unit
tables, rejected inputs) under the same three.  Each driver is built from
source here and reads a seeded batch written by the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2404_06452_amd import build as pkg_build
from paper_2404_06452_amd import chaingen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "san")
FIELDS = ("set_chain_off", "set_exec_off", "set_accel_off", "chain_cb_off", "cb_seg_off", "T",
          "D", "prio", "spin", "E", "exec", "A", "accel", "exec_core", "exec_prio",
          "accel_buckets", "accel_eps", "accel_kappa", "eps_hop")


def _write(cs, d):
    os.makedirs(d, exist_ok=True)
    np.array([cs.n_sets], np.int64).tofile(os.path.join(d, "n_sets.bin"))
    for f in FIELDS:
        np.ascontiguousarray(getattr(cs, f)).tofile(os.path.join(d, f + ".bin"))


def _batch(d, n=5000):
    p = chaingen.PRESETS["small_overheads"].replace(n_accel=2, max_seg_per_cb=2)
    _write(chaingen.generate(p, n), d)


def _run(exe, arg, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe, arg], capture_output=True, text=True, env=env, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "runtime error" not in report and "Sanitizer" not in report, report[-4000:]
    return report


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_oracle_under_sanitizers(tmp_path, san):
    d = str(tmp_path / "batch")
    _batch(d, 400)
    exe = str(tmp_path / "oracle_driver")
    src = [os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "paam_oracle.c"),
           os.path.join(ROOT, "oracle", "paam_des.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=all", "-fsanitize=" + san, "-o", exe] + src +
                          ["-lpthread"])
    out = _run(exe, d, {"ASAN_OPTIONS": "detect_leaks=0", "TSAN_OPTIONS": "halt_on_error=1"})
    assert "oracle driver ok" in out


@pytest.mark.skipif(not os.path.exists(pkg_build.hipcc()) and shutil.which("hipcc") is None,
                    reason="needs hipcc")
@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_host_library_under_sanitizers(tmp_path, san):
    d = str(tmp_path / "batch")
    _batch(d, 5000)       # >= 4096 sets: validation and packing run on several threads
    exe = str(tmp_path / "host_driver")
    srcs = [os.path.join(pkg_build.CSRC, s) for s in pkg_build.SOURCES]
    flags = [f for f in pkg_build.HIPCC_FLAGS if f not in ("-shared", "-O3")]
    host_san = []
    for s_ in san.split(","):
        host_san += ["-Xarch_host", "-fsanitize=" + s_]
    subprocess.check_call([pkg_build.hipcc()] + flags + ["-O1", "-g", "-fno-omit-frame-pointer"] +
                          host_san + ["-I", pkg_build.INCLUDE, "-I", pkg_build.CSRC, "-I", SAN,
                                      "-o", exe] + srcs + [os.path.join(SAN, "host_driver.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = _run(exe, d, {"ASAN_OPTIONS": "detect_leaks=0:protect_shadow_gap=0",
                        "TSAN_OPTIONS": "halt_on_error=1", "HIP_VISIBLE_DEVICES": ""})
    assert "host driver ok" in out
