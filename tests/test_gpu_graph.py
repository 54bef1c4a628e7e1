"""A plan step -- the re-plan from the advanced positions, spreading, and interpolation
with the position update -- captured once in a HIP graph and replayed: every replay, with
eager work and synchronisations between the replays, gives the bits of the same step run
eagerly, step after step along the advected trajectory, and exports between the replays
return the replayed update's plan arrays (every export recomputes on the stream)."""
import pytest
import torch

from paper_2012_06646_amd import workloads as wl
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_06646_amd import ibops
    return ibops


CASES = [(48, 60000, torch.float64, 0),     # shared spreading tiles, gathered interpolation
         (48, 60000, torch.float32, 0),
         (128, 1000000, torch.float64, 0),  # the benchmark's workload: LDS-tiled interpolation
         (48, 60000, torch.float64, 4)]     # walls along z: a fresh plan every step


KEYS = ("keys", "sorted_keys", "perm", "seg_off")


def exports(p):
    """Plan arrays of staggerings 0 and 1 (host copies)."""
    out = []
    for sid in (0, 1):
        e = p.export(sid)
        out.append([e[k].cpu() for k in KEYS] + [e["q"]])
    return out


def same_exports(a, b):
    return all(torch.equal(x, y) if torch.is_tensor(x) else x == y
               for ea, eb in zip(a, b) for x, y in zip(ea, eb))


@pytest.mark.parametrize("N,n,dtype,walls", CASES)
def test_captured_step_replays_match_eager(ib, N, n, dtype, walls):
    g = dict(wl.grid(3, N, 1.0), walls=walls)
    X0, F, u = wl.uniform_case(wl.grid(3, N, 1.0), n, 61)
    dt = 0.1 / N
    Fd, ud = to_dev(F, dtype), to_dev(u, dtype)
    steps = 5
    say(f"captured step N={N} n={n} dtype={dtype} walls={walls}")
    # the eager reference: step 0 from the positions, then advected re-plans
    pe = ib.Plan(g, n, dtype)
    Xe = to_dev(X0, dtype)
    ref = []
    for k in range(steps):
        if k == 0 or walls:
            pe.update(Xe)
        else:
            pe.update_advected()
        f = pe.spread(Fd)
        U = pe.interpolate_advect(ud, Xe, dt)
        ref.append((f.clone(), U.clone(), Xe.clone(), exports(pe)))
    del pe
    # step 0 eagerly, then one captured step replayed for steps 1 ..
    pg = ib.Plan(g, n, dtype)
    Xg = to_dev(X0, dtype)
    fg = torch.empty_like(ref[0][0])
    Ug = torch.empty_like(ref[0][1])
    pg.update(Xg)
    pg.spread(Fd, fg)
    pg.interpolate_advect(ud, Xg, dt, Ug)
    torch.cuda.synchronize()
    assert torch.equal(fg, ref[0][0]) and torch.equal(Ug, ref[0][1]) and torch.equal(Xg, ref[0][2])
    gr = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(gr, stream=cap):
            if walls:
                pg.update(Xg)  # walled plans re-plan from the positions
            else:
                pg.update_advected()
            pg.spread(Fd, fg)
            pg.interpolate_advect(ud, Xg, dt, Ug)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    for k in range(1, steps):
        gr.replay()
        other = (Fd * 2.0).abs().max()  # eager work between the replays
        torch.cuda.synchronize()
        assert float(other) > 0.0
        say(f"replay {k}")
        assert torch.equal(fg, ref[k][0]), f"replay {k}: spreading differs"
        assert torch.equal(Ug, ref[k][1]), f"replay {k}: interpolation differs"
        assert torch.equal(Xg, ref[k][2]), f"replay {k}: positions differ"
        assert same_exports(exports(pg), ref[k][3]), f"replay {k}: exports differ"
        assert same_exports(exports(pg), ref[k][3]), f"replay {k}: a second export differs"
    assert pg.status() == 0
