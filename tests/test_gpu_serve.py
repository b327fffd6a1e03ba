"""Serving loop: requests that arrive while others run are admitted by HBM
footprint and co-batched; every result must be bitwise the same as the
request solved alone through the plain path, and a request of each family
(Burgers, Euler) served in the mix must match the oracle stepped with the
same CFL time steps (1e-9, the multi-step parity bar)."""
import numpy as np
import pytest

import oracle

from paper_2004_08503_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08503_amd import idp_dg, serve
    return idp_dg, serve


def alone(idp_dg, req):
    sv = idp_dg.Solver(req.problem())
    u = W.initial_state_device(req)
    for _ in range(req.steps):
        sv.step_cfl(u, 0.5)
    out = u.cpu()
    sv.close()
    return out


@pytest.mark.parametrize("policy", ["ps", "srw"])
@pytest.mark.parametrize("budget_mb", [4096, 3], ids=["roomy", "one-at-a-time"])
def test_served_results_equal_alone(budget_mb, policy):
    idp_dg, serve = _mods()
    reqs = W.request_stream(10, rate=400.0, n_range=(4, 14), p_range=(2, 5),
                            steps_range=(3, 9), seed=11)
    # srw: a small tick budget, so that requests pause and resume
    srv = serve.Server(hbm_budget=budget_mb * 2 ** 20, keep_results=True, policy=policy,
                       max_active_nodes=0 if policy == "srw" else 1 << 21, tick_nodes=3000)
    done = srv.run(reqs)
    assert [d.rid for d in done] == [r.rid for r in reqs]
    # admission counted what a request really holds (state, handle workspace,
    # alignment slack), and never more than the budget at once
    assert srv.peak_used <= budget_mb * 2 ** 20
    for r in reqs:
        prob = r.problem()
        sv = idp_dg.Solver(prob, workspace=True)
        held = sv._ws.numel() + 8 * prob.nc * prob.num_nodes
        sv.close()
        assert serve.footprint_bytes(r) == held
    for d, r in zip(done, reqs):
        assert d.finished >= d.arrival - 1e-3
        assert torch.equal(d.result, alone(idp_dg, r)), r
    s = serve.summarize(done)
    assert s["tts_s_p99"] >= s["tts_s_p50"] > 0


def test_served_results_match_the_oracle():
    idp_dg, serve = _mods()
    reqs = W.request_stream(8, rate=600.0, n_range=(4, 10), p_range=(2, 4),
                            steps_range=(3, 8), seed=23)
    kinds = {r.kind for r in reqs}
    assert kinds == {"euler", "burgers"}
    done = serve.Server(hbm_budget=4096 * 2 ** 20, keep_results=True).run(reqs)
    checked = set()
    for d, r in zip(done, reqs):
        if r.kind in checked:
            continue
        checked.add(r.kind)
        prob = r.problem()
        ref = W.initial_state_device(r).cpu().numpy()
        for _ in range(r.steps):
            ref = oracle.step(prob, ref, 0.5 * oracle.max_dt(prob, ref))
        got = d.result.numpy().reshape(ref.shape)
        err = (np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max()
        print("served %s %d^2 p=%d, %d steps: max relative error %.2e" % (r.kind, r.n, r.p, r.steps, err))
        assert err <= 1e-9, (r, err)
    assert checked == kinds


@pytest.mark.parametrize("caps", [dict(max_active_nodes=700), dict(max_active=1), dict(max_active_nodes=0),
                                  dict(max_active_nodes=700, small_nodes=300),
                                  dict(max_active_nodes=700, small_nodes=0)],
                         ids=["node-cap", "one-active", "no-cap", "small-class", "strict-order"])
def test_admission_caps_keep_results(caps):
    """Admission by node count or request count only changes when requests
    run, not what they compute."""
    idp_dg, serve = _mods()
    reqs = W.request_stream(8, rate=800.0, n_range=(4, 12), p_range=(2, 4),
                            steps_range=(3, 7), seed=19)
    done = serve.Server(hbm_budget=4096 * 2 ** 20, keep_results=True, **caps).run(reqs)
    assert [d.rid for d in done] == [r.rid for r in reqs]
    for d, r in zip(done, reqs):
        assert torch.equal(d.result, alone(idp_dg, r)), r


def test_fifo_plain_matches():
    idp_dg, serve = _mods()
    reqs = W.request_stream(4, rate=1000.0, n_range=(4, 8), p_range=(2, 3),
                            steps_range=(2, 4), seed=3)
    done = serve.run_fifo_plain(reqs, keep_results=True)
    for d, r in zip(done, reqs):
        assert torch.equal(d.result, alone(idp_dg, r))


def test_small_requests_pass_a_waiting_large_one():
    """With a node cap that lets one large request run at a time, a small
    request that arrives behind a second, waiting large one is admitted
    before it (small requests do not wait their turn in arrival order), and
    every result still equals the request solved alone."""
    idp_dg, serve = _mods()
    from paper_2004_08503_amd.workloads import Request
    reqs = [Request(rid=0, kind="euler", n=24, p=3, steps=40, arrival=0.0, seed=1),
            Request(rid=1, kind="euler", n=24, p=3, steps=10, arrival=0.0, seed=2),
            Request(rid=2, kind="burgers", n=6, p=2, steps=5, arrival=0.0, seed=3)]
    big = reqs[0].problem().num_nodes
    small = reqs[2].problem().num_nodes
    assert small < big // 16
    srv = serve.Server(hbm_budget=4096 * 2 ** 20, keep_results=True, max_active_nodes=big, small_nodes=big // 16)
    done = srv.run(reqs)
    by = {d.rid: d for d in done}
    assert by[2].admitted <= by[1].admitted          # passed the waiting large request
    assert by[1].admitted >= by[0].admitted
    assert by[2].finished < by[0].finished           # ran beside the first large one
    for d, r in zip(done, reqs):
        assert torch.equal(d.result, alone(idp_dg, r)), r


def test_request_over_the_budget_is_an_error():
    """A request whose footprint exceeds the whole HBM budget can never be
    admitted: the server says so instead of waiting for ever."""
    idp_dg, serve = _mods()
    reqs = W.request_stream(2, rate=1000.0, n_range=(32, 32), p_range=(3, 3), steps_range=(2, 2), seed=4)
    budget = serve.footprint_bytes(reqs[0]) - 1
    with pytest.raises(ValueError, match="more than the HBM budget"):
        serve.Server(hbm_budget=budget).run(reqs)
