"""The device code of libibops, compiled for gfx950 here (no GPU needed): its atomic
instructions are all integer ones.  Spreading sums in fixed point with integer LDS adds, and
the plan's counters, histograms and flags are integers, so no floating-point atomic (whose
result would depend on the order of work) appears anywhere."""
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2012_06646_amd import build as B

# every read-modify-write mnemonic: global/flat/buffer atomics and LDS atomics
RMW = re.compile(r"^\s*((?:global|flat|buffer)_atomic_\w+|ds_(?:add|sub|rsub|min|max|inc|dec|and|or|xor|"
                 r"pk_add|cmpst|cmpswap|wrxchg|cond_sub|sub_clamp)\w*)", re.M)
INTEGER_RMW = re.compile(r"^(ds_(add|max)(_rtn)?_u(32|64)|(global|flat)_atomic_(add|or|umax)(_x2)?)$")
FLOAT_SUFFIX = re.compile(r"_(f16|bf16|f32|f64)\b")


def device_asm(src, out):
    cmd = [B.HIPCC] + [f for f in B.FLAGS if f != "-fPIC"] + ["--cuda-device-only", "-S", "-x", "hip",
                                                             os.path.join(B.CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    with open(out) as fh:
        return fh.read()


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if shutil.which(B.HIPCC) is None and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("asm")
    srcs = [s for s in B.SOURCES if s.endswith(".hip")]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        texts = list(ex.map(lambda s: device_asm(s, str(d / (s + ".s"))), srcs))
    return dict(zip(srcs, texts))


def test_no_floating_point_atomics(asm):
    seen = {}
    for src, text in asm.items():
        for m in RMW.findall(text):
            seen.setdefault(m, set()).add(src)
    assert seen, "no atomics found: the pattern no longer matches the assembly"
    assert "ds_add_u64" in seen  # the fixed-point spreading sums
    floats = {m: s for m, s in seen.items() if FLOAT_SUFFIX.search(m)}
    assert not floats, floats
    others = {m: s for m, s in seen.items() if not INTEGER_RMW.match(m)}
    assert not others, others
