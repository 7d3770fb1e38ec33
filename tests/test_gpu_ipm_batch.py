"""Solvers stepped in lockstep with batched condensation and solve
(rh_ipm_batch_step) take exactly the iterations of the same solvers stepped
one by one (rh_ipm_step), and end at the same points bit for bit."""
import numpy as np
import pytest

import synthnet

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _api():
    from paper_2203_11875_amd import api
    return api


def _nets():
    base = synthnet.case9(1)
    return [base, synthnet.scale_loads(base, 1), synthnet.case118(0),
            synthnet.scale_loads(synthnet.case118(0), 2)]


def test_lockstep_equals_one_by_one():
    api = _api()
    nets = _nets()
    print("ipm batch: 2 x syn9 + 2 x syn118 scenarios", flush=True)
    # one by one
    single = []
    for net in nets:
        G = api.Net(net)
        ipm = api.Ipm(G, tol=1e-6)
        log = []
        for _ in range(200):
            code, info = ipm.step()
            assert code == 0, (code, info)
            log.append(info)
            if info["converged"]:
                break
        st = {k: v.cpu().numpy() for k, v in ipm.state().items()}
        single.append((log, st))
        ipm.close()
        G.close()
    # lockstep, every handle on its own stream
    Gs = [api.Net(net, stream=torch.cuda.Stream()) for net in nets]
    ipms = [api.Ipm(G, tol=1e-6) for G in Gs]
    B = api.Batch(Gs, stream=torch.cuda.Stream())
    IB = api.IpmBatch(B, ipms)
    logs = [[] for _ in nets]
    done = [False] * len(nets)
    for _ in range(200):
        res = IB.step()
        for i, (code, info) in enumerate(res):
            if done[i]:
                assert info["converged"] == 1
                continue
            assert code == 0, (i, code, info)
            logs[i].append(info)
            done[i] = bool(info["converged"])
        if all(done):
            break
    assert all(done)
    for i, (log, st) in enumerate(single):
        assert len(logs[i]) == len(log), i
        for a, b in zip(logs[i], log):
            for key in ("mu", "alpha_pr", "alpha_du", "delta_w", "obj", "ls_trials", "err"):
                assert a[key] == b[key], (i, key, a[key], b[key])
        got = {k: v.cpu().numpy() for k, v in ipms[i].state().items()}
        for k in st:
            assert np.array_equal(got[k], st[k]), (i, k)
    # the instances need different iteration counts, so some idled
    assert len({len(l) for l in logs}) > 1


def test_batch_step_rejects_mismatched_solver():
    api = _api()
    nets = _nets()[:2]
    Gs = [api.Net(n) for n in nets]
    ipms = [api.Ipm(Gs[1]), api.Ipm(Gs[0])]        # swapped
    B = api.Batch(Gs)
    with pytest.raises(api.RhError):
        api.IpmBatch(B, ipms).step()


def test_batch_backward_needs_converged_solvers():
    api = _api()
    nets = _nets()[:2]
    Gs = [api.Net(n) for n in nets]
    ipms = [api.Ipm(G, tol=1e-8) for G in Gs]
    B = api.Batch(Gs)
    with pytest.raises(api.RhError) as e:
        api.IpmBatch(B, ipms).backward(None, None, torch.ones(2, dtype=torch.float64,
                                                              device="cuda"))
    assert e.value.code == -5


def test_batch_rebinds_new_solvers():
    """A batch stepped with one set of solvers, then (after those are closed)
    with new ones, steps the new ones from their own starting points: the
    binding follows the solvers, not the addresses they happen to get."""
    api = _api()
    nets = _nets()[:2]
    Gs = [api.Net(n) for n in nets]
    B = api.Batch(Gs)
    first = [api.Ipm(G, tol=1e-6) for G in Gs]
    IB = api.IpmBatch(B, first)
    for _ in range(3):
        IB.step()
    for p in first:
        p.close()
    second = [api.Ipm(G, tol=1e-6) for G in Gs]
    got = api.IpmBatch(B, second).step()
    for i, G in enumerate(Gs):
        ref = api.Ipm(G, tol=1e-6)
        code, info = ref.step()
        assert got[i][0] == code == 0
        for key in ("mu", "alpha_pr", "alpha_du", "obj", "err"):
            assert got[i][1][key] == info[key], (i, key)
        s1 = {k: v.cpu().numpy() for k, v in second[i].state().items()}
        s2 = {k: v.cpu().numpy() for k, v in ref.state().items()}
        for k in s1:
            assert np.array_equal(s1[k], s2[k]), (i, k)
        ref.close()
