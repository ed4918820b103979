"""Serving loop: results identical alone and mixed, admission within the
HBM budget (GPU), and the trace and summary logic (CPU)."""
import threading

import numpy as np
import pytest

from paper_1408_4675_amd import scenarios as sc
from paper_1408_4675_amd.serving import Result, summarize


def test_trace_is_poisson_with_the_requested_sizes():
    reqs = sc.serving_trace(seed=3, n_requests=400, rate=20.0, sizes=(32, 48), medium_pool=2,
                            steps_range=(5, 9))
    t = np.array([r.arrival for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1 / 20.0) < 0.15 / 20.0          # mean inter-arrival 50 ms
    assert {r.scenario.grid.nx for r in reqs} == {32, 48}
    assert all(5 <= r.scenario.steps <= 9 for r in reqs)
    # pooled media are shared, amplitudes are per request
    same = [r for r in reqs if r.scenario.grid.nx == 32]
    ids = {id(r.scenario.medium.c0) for r in same}
    assert len(ids) <= 2
    amps = {float(r.scenario.source.amp[0]) for r in same}
    assert len(amps) == len(same)


def test_summary_percentiles():
    rs = [Result(i, 100, 10, arrival=float(i), start=float(i), finish=float(i) + 1.0 + i * 0.01)
          for i in range(101)]
    s = summarize(rs)
    assert s["requests"] == 101
    assert abs(s["p50_latency_s"] - 1.5) < 1e-9
    assert abs(s["p99_latency_s"] - 1.99) < 1e-9
    assert abs(s["makespan_s"] - (100 + 2.0)) < 1e-9
    assert abs(s["point_updates_per_s"] - 101 * 1000 / 102.0) < 1e-9


@pytest.mark.gpu
def test_live_simulations_have_distinct_streams():
    """torch.cuda.Stream() hands out one of 32 pooled streams per device in
    turn, so the 33rd is the 1st again; a Simulation takes a HIP stream of its
    own, so 34 simulations alive at once run on 34 streams, and each still
    gives the result it gives alone."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4675_amd.simulation import Simulation
    print("\n[case] 34 live 16^3 simulations, stream handles", flush=True)
    pool = [torch.cuda.Stream() for _ in range(33)]
    assert pool[0].cuda_stream == pool[32].cuda_stream          # the pooled streams repeat
    scen = sc.small_case(16, 16, 16, seed=4, steps=6)
    sims = [Simulation(scen, tune=False) for _ in range(34)]
    try:
        handles = [s.stream.cuda_stream for s in sims]
        assert len(set(handles)) == len(sims)
        assert not set(handles) & {p.cuda_stream for p in pool}
        for s in sims:
            s.step(scen.steps)
        outs = [s.gather(sc.REC_P_MAX, device=False) for s in sims]
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
    finally:
        for s in sims:
            s.close()


@pytest.mark.gpu
def test_mixed_results_equal_alone_and_budget_holds():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4675_amd.serving import Server, run_fifo
    from paper_1408_4675_amd.simulation import workspace_size
    reqs = sc.serving_trace(seed=5, n_requests=8, rate=400.0, sizes=(32, 48, 64),
                            medium_pool=2, steps_range=(20, 60))
    print("\n[case] serving: 8 requests of 32^3-64^3, mixed vs alone", flush=True)
    alone = {r.rid: r for r in run_fifo(reqs, keep_outputs=True)}
    foot = max(workspace_size(r.scenario) for r in reqs)
    # host preparation in two worker threads (no device calls there); every
    # device call in this thread
    srv = Server(budget_bytes=2 * foot + 1, max_active=4, chunk_steps=16, keep_outputs=True,
                 prepare_workers=2)
    mixed = srv.run(reqs)
    assert srv.peak_used <= 2 * foot + 1
    assert srv.peak_active >= 2
    assert len(mixed) == len(reqs)
    for r in mixed:
        a = alone[r.rid]
        assert set(r.outputs) == set(a.outputs) and r.outputs
        for k in r.outputs:
            assert np.array_equal(r.outputs[k], a.outputs[k]), (r.rid, k)


def test_scheduler_admission_budget_and_chunks(monkeypatch):
    """The scheduler alone, on a stand-in for the simulation (no GPU): requests
    are admitted in arrival order within the footprint budget and the slot
    limit, every request runs exactly its steps in chunks, and each finishes.
    The host preparation (the library's kw_prepare, which makes no device
    call) runs in worker threads; the device set-up only in the scheduling
    thread."""
    import paper_1408_4675_amd.serving as S
    from paper_1408_4675_amd.simulation import workspace_size as real_workspace_size

    log = {"active": 0, "peak": 0, "steps": {}, "order": [], "prepare_threads": set()}

    main_thread = threading.get_ident()

    class RecordingPrepared(S.Prepared):
        # the real host-only preparation (kw_prepare runs on the CPU), noting its thread
        def __init__(self, scen):
            log["prepare_threads"].add(threading.get_ident())
            super().__init__(scen)

    class FakeSim:
        def __init__(self, scen, device="cuda", prepared=None):
            assert threading.get_ident() == main_thread      # device set-up: scheduling thread only
            assert isinstance(prepared, S.Prepared) and prepared.handle
            assert prepared.workspace_bytes == real_workspace_size(scen)
            self.scen = scen
            self.stream = None
            log["active"] += 1
            log["peak"] = max(log["peak"], log["active"])
            log["order"].append(scen.name)

        def step(self, n):
            log["steps"][self.scen.name] = log["steps"].get(self.scen.name, 0) + n

        def gather(self, what, device=False):
            return np.zeros(1, np.float32)

        def close(self):
            log["active"] -= 1

    class FakeEvent:
        def record(self, stream):
            pass

        def query(self):
            return True

    reqs = sc.serving_trace(seed=2, n_requests=12, rate=1e6, sizes=(32, 48), medium_pool=1,
                            steps_range=(5, 40))
    for i, r in enumerate(reqs):
        r.scenario.name = "r%d" % i
    foot = {id(r.scenario): (100 if r.scenario.grid.nx == 32 else 250) for r in reqs}
    monkeypatch.setattr(S, "Simulation", FakeSim)
    monkeypatch.setattr(S, "Prepared", RecordingPrepared)
    monkeypatch.setattr(S, "workspace_size", lambda scen: foot[id(scen)])
    monkeypatch.setattr(S.torch.cuda, "Event", FakeEvent)
    srv = S.Server(budget_bytes=600, max_active=3, chunk_steps=16)
    res = srv.run(reqs)
    assert len(res) == 12 and log["active"] == 0
    assert log["order"] == ["r%d" % i for i in range(12)]          # arrival order
    assert srv.peak_active <= 3 and log["peak"] <= 3
    assert srv.peak_used <= 600
    assert log["prepare_threads"] and main_thread not in log["prepare_threads"]
    for i, r in enumerate(reqs):
        assert log["steps"]["r%d" % i] == r.scenario.steps
    with pytest.raises(ValueError):
        S.Server(budget_bytes=50, max_active=3).run(reqs)            # a request above budget
