"""Checks on the gfx950 code of the library's kernels, on the CPU: each HIP
source is compiled to device assembly with the build's own flags, and the
kernels must hold

* no flat atomics: the LDS tables of the analysis and feature kernels reach
  their helpers through plain pointers, and only code the compiler can see
  through (inlined) gets LDS atomics; an outlined helper turns them into flat
  atomics, which LDS does not take for fp64;
* no calls (every helper inlined, for the same reason);
* no packed fp32 arithmetic (the build disables it; some of its forms have
  given wrong results without an error)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2404_06452_amd import build as pkg_build

SOURCES = [s for s in pkg_build.SOURCES if s.endswith(".hip")]


def _device_asm(tmp_path, src):
    hipcc = pkg_build.hipcc()
    if shutil.which(hipcc) is None and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    flags = [f for f in pkg_build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    out = os.path.join(str(tmp_path), src + ".s")
    cmd = [hipcc] + flags + ["--cuda-device-only", "-S", "-I", pkg_build.INCLUDE, "-I",
                             pkg_build.CSRC, "-o", out, os.path.join(pkg_build.CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    with open(out) as f:
        return f.read()


def _kernel_bodies(asm):
    """Instruction lines of every function in the assembly, by symbol."""
    bodies, cur = {}, None
    for line in asm.split("\n"):
        m = re.match(r"^(_Z\S+):", line)
        if m:
            cur = m.group(1)
            bodies[cur] = []
            continue
        if cur is not None:
            if line.startswith(".Lfunc_end"):
                cur = None
                continue
            ins = line.strip()
            if ins and not ins.startswith((";", ".")):
                bodies[cur].append(ins.split()[0])
    return bodies


@pytest.mark.parametrize("src", SOURCES)
def test_kernels_have_no_flat_atomics_calls_or_packed_fp32(tmp_path, src):
    bodies = _kernel_bodies(_device_asm(tmp_path, src))
    assert bodies, "no functions found in the assembly of " + src
    for name, ops in bodies.items():
        flat_atomics = sorted({o for o in ops if o.startswith("flat_atomic")})
        assert not flat_atomics, (name, flat_atomics)
        assert "s_swappc_b64" not in ops, (name, "calls a function")
        packed = sorted({o for o in ops if re.match(r"v_pk_(add|mul|fma)_f32", o)})
        assert not packed, (name, packed)
