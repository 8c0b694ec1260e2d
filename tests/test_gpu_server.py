"""GPU serving loop: admission by the pool budget, continuous batching and
retirement; every result equals its box stepped alone (bitwise)."""
import numpy as np
import pytest

try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

import fish_inputs as fi
from oracle import OUTFLOW, PERIODIC

pytestmark = pytest.mark.gpu

FIELDS = ("cell", "bx", "by", "bz")

# (shape, bc, nsteps, seed)
REQS = [
    ((16, 16, 16), (PERIODIC,) * 3, 5, 11),
    ((24, 20, 12), (PERIODIC,) * 3, 2, 12),
    ((9, 30, 5), (PERIODIC,) * 3, 7, 13),
    ((11, 7, 6), (OUTFLOW,) * 3, 3, 14),
    ((20, 20, 20), (PERIODIC,) * 3, 4, 15),
    ((12, 10, 18), (PERIODIC, OUTFLOW, PERIODIC), 6, 16),
]


def _state(n, seed):
    return fi.random_fourier_state(n, seed=seed, mach=0.6, beta=5.0, kmax=2)


def _alone(n, bc, st, prec, steps):
    import paper_0910_2854_amd as fish
    g = fish.Box(*n, precision=prec, bc=bc)
    g.set_state(st)
    for _ in range(steps):
        g.strang_step(0.0)
    out = g.get_state()
    g.close()
    return out


@pytest.mark.parametrize("prec,graph", [("fp32", False), ("fp32", True), ("fp64", False)])
def test_server_results_equal_alone_and_admission_waits_for_room(prec, graph):
    import paper_0910_2854_amd as fish
    print(f"server {prec} graph={graph}: {len(REQS)} requests", flush=True)
    # room for the two largest boxes at a time only: admission must wait
    need = sorted(fish.box_pool_bytes(n, prec, bc=bc) for n, bc, _, _ in REQS)
    srv = fish.Server(need[-1] + need[-2] + 1024, chunk_steps=2, precision=prec)
    srv.use_graph(graph)
    for tag, (n, bc, k, seed) in enumerate(REQS):
        srv.submit(tag, _state(n, seed), k, bc=bc)
    done = {}
    max_resident = 0
    for _ in range(200):
        for tag, status, out in srv.pump():
            assert status == fish.FISH_OK, tag
            done[tag] = out
        st = srv.stats()
        max_resident = max(max_resident, st["resident"])
        if len(done) == len(REQS):
            break
    assert len(done) == len(REQS)
    assert 1 <= max_resident < len(REQS)
    for tag, (n, bc, k, seed) in enumerate(REQS):
        ref = _alone(n, bc, _state(n, seed), prec, k)
        for f in FIELDS:
            assert np.array_equal(done[tag][f], ref[f]), (tag, f)
    assert srv.stats()["resident"] == 0 and srv.stats()["queued"] == 0
    srv.close()


def test_server_refuses_a_request_larger_than_the_pool():
    import paper_0910_2854_amd as fish
    print("server oversized request", flush=True)
    srv = fish.Server(fish.box_pool_bytes((8, 8, 8), "fp32"), precision="fp32")
    with pytest.raises(fish.FishError) as e:
        srv.submit(0, _state((16, 16, 16), 1), 2)
    assert e.value.code == fish.FISH_ERR_NOMEM
    srv.close()


def test_server_completes_a_bad_request_with_its_status():
    import paper_0910_2854_amd as fish
    print("server bad request", flush=True)
    srv = fish.Server(64 << 20, precision="fp64")
    bad = fi.uniform_state((6, 6, 6), p=0.5)
    bad["cell"][0, 1, 1, 1] = -1.0
    srv.submit(7, bad, 3)
    srv.submit(8, _state((8, 8, 8), 2), 1)
    got = {}
    for _ in range(10):
        for tag, status, out in srv.pump():
            got[tag] = status
        if len(got) == 2:
            break
    assert got == {7: fish.FISH_ERR_STATE, 8: fish.FISH_OK}
    srv.close()


@pytest.mark.timeout(600)
def test_server_full_size_requests_equal_alone():
    """The serving workload the benchmark times, at full size: 12 requests of
    its saturated mix (edges 32-192, 10-200 double steps, Mach 0.5, beta 10),
    all queued at once into a server with the benchmark's settings (FP32,
    graph replays, chunks of 5 steps); every completed request's state is
    bitwise its box stepped alone the same number of steps."""
    import paper_0910_2854_amd as fish
    reqs = fi.serving_requests(12, rate=1.0, seed=7)

    def state(r):
        e = r["edge"]
        return fi.random_fourier_state((e, e, e), seed=r["seed"], mach=0.5, beta=10.0, kmax=4)

    print(f"server full size: edges {[r['edge'] for r in reqs]}, steps {[r['steps'] for r in reqs]}", flush=True)
    states = [state(r) for r in reqs]
    pool = sum(fish.box_pool_bytes((r["edge"],) * 3, "fp32") for r in reqs) + (64 << 20)
    srv = fish.Server(pool, chunk_steps=5, max_boxes=4096, precision="fp32")
    srv.use_graph(True)
    for tag, r in enumerate(reqs):
        srv.submit(tag, states[tag], r["steps"])
    done = {}
    for _ in range(1000):
        for tag, status, out in srv.pump():
            done[tag] = (status, out)
        if len(done) == len(reqs):
            break
    srv.close()
    assert len(done) == len(reqs)
    for tag, r in enumerate(reqs):
        e = r["edge"]
        print(f"  request {tag}: edge {e}, {r['steps']} steps", flush=True)
        g = fish.Box(e, e, e, precision="fp32")
        g.set_state(states[tag])
        for _ in range(r["steps"]):
            g.strang_step(0.0)
        status, out = done[tag]
        if status != fish.FISH_OK:
            with pytest.raises(fish.FishError):
                g.get_state()
            g.close()
            continue
        ref = g.get_state()
        g.close()
        for k in FIELDS:
            assert np.array_equal(out[k], ref[k]), (tag, k)
