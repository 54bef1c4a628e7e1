"""Plan tunings (ib_tuning) and the autotuner: every tuning gives the same plan arrays and
operator values within tolerance of the oracle; the tuner's choice is cached and found."""
import json

import numpy as np
import pytest
import torch

from paper_2012_06646_amd import workloads as wl
from tests.gpu_util import TOL, normwise, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_06646_amd import ibops
    return ibops


TUNINGS = [None, {"spread_tile": 1}, {"spread_tile": 2}, {"spread_tile": 3}, {"split_points": 256},
           {"split_points": -1}, {"radix_bits": 8}, {"radix_bits": 4},
           {"spread_tile": 3, "split_points": 512, "radix_bits": 6}]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_every_tuning_matches_oracle(ib, orc, dtype):
    g = wl.grid(3, [40, 36, 44], 1.0)
    X, F, u = wl.uniform_case(g, 60000, 51)
    nd = np.float64 if dtype == torch.float64 else np.float32
    Xc, Fc, uc = X.astype(nd), F.astype(nd), u.astype(nd)
    f_ref = orc.spread(g, Xc.astype(np.float64), Fc.astype(np.float64))
    U_ref = orc.interp(g, Xc.astype(np.float64), uc.astype(np.float64))
    ref_plan = ref_vals = None
    for t in TUNINGS:
        p = ib.Plan(g, X.shape[0], dtype, tuning=t).update(to_dev(Xc, dtype))
        f = to_host(p.spread(to_dev(Fc, dtype)))
        U = to_host(p.interpolate(to_dev(uc, dtype)))
        ef, eU = normwise(f, f_ref), normwise(U, U_ref)
        say(f"tuning {t}: spread {ef:.2e} interp {eU:.2e}")
        assert ef <= TOL[dtype] and eU <= TOL[dtype]
        # the fixed-point scale depends on the forces and the largest cell count only, and
        # integer sums on nothing else: every tuning gives the same bits
        if ref_vals is None:
            ref_vals = (f, U)
        assert np.array_equal(f, ref_vals[0]) and np.array_equal(U, ref_vals[1]), f"tuning {t}"
        e = p.export(0)
        arrays = [to_host(e[k]) for k in ("keys", "sorted_keys", "perm", "seg_off")]
        if ref_plan is None:
            ref_plan = arrays
        for a, b in zip(arrays, ref_plan):
            assert np.array_equal(a, b)


def test_autotune_caches_and_plan_finds_it(ib, tmp_path, monkeypatch):
    from paper_2012_06646_amd import tune
    monkeypatch.setenv("IB_TUNE_CACHE", str(tmp_path / "tune.json"))
    dtype = torch.float32
    g = wl.grid(3, 32, 1.0)
    X, F, u = wl.uniform_case(g, 150000, 53)
    Xd, Fd, ud = to_dev(X, dtype), to_dev(F, dtype), to_dev(u, dtype)
    best, timings = tune.autotune(g, Xd, Fd, ud, reps=3)
    say(f"autotune best {best} over {len(timings)} candidates")
    assert len(timings) >= 3 and "(0, 0, 0)" in timings  # distinct layouts only
    data = json.load(open(tmp_path / "tune.json"))
    entry = data[tune.key(g, dtype, X.shape[0])]
    # the stored times come from different rounds of interleaved timing (the winner of an
    # axis is timed again with the next axis), so they compare within the timing noise
    assert entry["tuning"] == best and entry["ms"] <= 1.1 * entry["default_ms"]
    p = ib.Plan(g, X.shape[0], dtype, tuning="auto")
    assert p.tuning == best
    p.update(Xd)
    f1 = p.spread(Fd)
    f0 = ib.Plan(g, X.shape[0], dtype).update(Xd).spread(Fd)
    assert normwise(to_host(f1), to_host(f0).astype(np.float64)) <= TOL[dtype]
