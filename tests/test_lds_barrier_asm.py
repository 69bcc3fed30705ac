"""The line FFT's LDS exchanges keep their reads between the two barriers
that enclose them (CPU-only: compiles a probe kernel to gfx950 assembly).

Each non-final pass writes its outputs to LDS, waits at a barrier, reads its
next inputs and waits again before the next pass may overwrite LDS.  The
compiler treats the barrier as a side effect that writes no memory and may
sink the reads below the closing barrier into a conditional block (seen with
a fused transform whose store depends on a per-workgroup flag); other waves
then overwrite the data before those reads run.  The exchange barrier carries
an empty asm that clobbers memory to prevent this; the test checks the
assembly: between two barriers of a transform there is always an LDS access.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_03585_amd", "csrc")
PROBE = os.path.join(ROOT, "tests", "asm_probe", "lds_exchange_probe.hip")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def compile_probe(include_dir, out_dir):
    out = os.path.join(out_dir, "probe.s")
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-I", include_dir,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--cuda-device-only", "-S", PROBE, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return open(out).read()


def empty_barrier_pairs(asm):
    """Per kernel: (barrier count, number of consecutive barrier pairs with
    no LDS instruction between them)."""
    res = {}
    for m in re.finditer(r"^(_Z\S+):[^\n]*\n(.*?)^\.Lfunc_end", asm, re.S | re.M):
        lines = [l.strip() for l in m.group(2).split("\n")]
        bars = empty = 0
        lds_since = True
        for l in lines:
            if l.startswith("s_barrier"):
                bars += 1
                empty += not lds_since
                lds_since = False
            elif l.startswith("ds_"):
                lds_since = True
        res[m.group(1)] = (bars, empty)
    return res


def test_exchange_reads_stay_between_barriers(tmp_path):
    res = empty_barrier_pairs(compile_probe(CSRC, str(tmp_path)))
    # 4096 = 16^3: three passes, two exchanges per transform; 16384 = 16^3 x 4:
    # three exchanges per transform; two barriers per exchange
    want = {"4096": 8, "16384": 12}
    assert len(res) == 2
    for name, (bars, empty) in res.items():
        n = re.search(r"ILi(\d+)E", name).group(1)
        assert bars == want[n], (name, bars)
        assert empty == 0, f"{name}: LDS reads moved past an exchange barrier"


def test_probe_detects_reads_moved_without_the_clobber(tmp_path):
    """Sensitivity of the check: the same header with a plain barrier (no
    memory clobber) lets this compiler move the reads, and the scan sees it."""
    src = open(os.path.join(CSRC, "fft_line.hpp")).read()
    plain = src.replace('asm volatile("" ::: "memory");', "", 1)
    assert plain != src
    d = tmp_path / "plain"
    d.mkdir()
    (d / "fft_line.hpp").write_text(plain)
    res = empty_barrier_pairs(compile_probe(str(d), str(tmp_path)))
    if not any(e for _, e in res.values()):
        pytest.skip("this compiler keeps the reads in place even without the clobber")
    assert any(e for _, e in res.values())
