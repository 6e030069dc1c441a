"""Graph capture of the sweep: every replay equals the eager call it
records, also with eager work and synchronisations between replays."""
import numpy as np
import pytest
import torch

from synth import workloads as wl

from gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_batched_graph_replays_match_eager():
    from paper_2205_04295_amd import api, graph
    specs = [dict(seed=131, H=192, N=64, M=2, J=6), dict(seed=132, H=320, N=128, M=3, J=4),
             dict(seed=133, H=512, N=256, M=1, J=3)]
    ws = [wl.small_case(name=f"g{i}", **s) for i, s in enumerate(specs)]
    prm = dict(ws[0].params, iterations=1)
    jobs_g = [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"]) for d in map(to_dev, ws)]
    jobs_e = [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"]) for d in map(to_dev, ws)]
    g = graph.capture_batched(jobs_g, **prm)
    for rep in range(3):
        g.replay()
        api.rpie_batched(jobs_e, **prm)
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        for a, b in zip(jobs_g, jobs_e):
            assert torch.equal(a["obj"], b["obj"]), rep
            assert torch.equal(a["probe"], b["probe"]), rep
        del junk


def test_batched_graph_lanes_of_uneven_jobs():
    """44 jobs of uneven scan length captured as one launch chain: the driver
    deals them to 36 launch lanes, so 8 jobs start when the shorter job ahead
    of them in their lane has taken its last update.  Every replay equals
    the eager call (two streams of 22 jobs, one lane each) bitwise, error
    curves included, and each job matches its plain sweep to float rounding
    after the first."""
    from paper_2205_04295_amd import api, graph
    from gpu_util import rel_l2, run_gpu
    specs = []
    for i in range(44):
        N = (64, 64, 128, 128)[i % 4]
        specs.append(dict(seed=150 + i, H=N + 64, N=N, M=1 + (i // 4) % 3, J=2 + (5 * i) % 11))
    ws = [wl.small_case(name=f"l{i}", **s) for i, s in enumerate(specs)]
    prm = dict(ws[0].params, iterations=1)

    def jobs():
        return [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"],
                     err=torch.zeros(1, dtype=torch.float32, device="cuda:0")) for d in map(to_dev, ws)]
    jobs_g, jobs_e = jobs(), jobs()
    g = graph.capture_batched(jobs_g, **prm)
    for rep in range(3):
        g.replay()
        api.rpie_batched(jobs_e, **prm)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(jobs_g, jobs_e)):
            assert torch.equal(a["obj"], b["obj"]), (rep, k)
            assert torch.equal(a["probe"], b["probe"]), (rep, k)
            assert torch.equal(a["err"], b["err"]), (rep, k)
        if rep == 0:
            for w, j in zip(ws, jobs_g):
                r = run_gpu(w, prm)
                assert rel_l2(j["obj"].cpu().numpy(), r["O"]) < 1e-5
                assert rel_l2(j["probe"].cpu().numpy(), r["P"]) < 1e-5
                assert np.allclose(j["err"].cpu().numpy(), r["err"], rtol=1e-5, atol=0)


def test_plain_graph_replays_match_eager():
    from paper_2205_04295_amd import api, graph
    w = wl.small_case(141, 320, 128, 2, 8, name="gp")
    prm = dict(w.params, iterations=1)
    dg, de = to_dev(w), to_dev(w)
    eg = torch.zeros(1, dtype=torch.float32, device="cuda")
    ee = torch.zeros(1, dtype=torch.float32, device="cuda")
    api.rpie(de["obj"].clone(), de["probe"].clone(), de["pos"], de["I"], **prm)  # kernel attributes
    g, ws = graph.capture_plain(dg["obj"], dg["probe"], dg["pos"], dg["I"], err=eg, **prm)
    for rep in range(3):
        g.replay()
        api.rpie(de["obj"], de["probe"], de["pos"], de["I"], err=ee, **prm)
        torch.cuda.synchronize()
        assert torch.equal(dg["obj"], de["obj"]) and torch.equal(dg["probe"], de["probe"]), rep
        assert torch.equal(eg, ee)
