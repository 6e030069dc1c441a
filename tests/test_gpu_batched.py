"""Batched M-rPIE: independent reconstructions of uneven N, M, J advanced
lock-step in shared launches must each match the plain sweep of the same job
to float rounding (the single-job column pass keeps its first and last FFT
stages in registers, and a single small job runs the one-workgroup LDS sweep
while batches run it through the passes; jobs on the same kernels are
bitwise equal), and the oracle to the plain sweep's tolerance."""
import numpy as np
import pytest
import torch

from synth import workloads as wl

from gpu_util import need_gpu, rel_l2, run_gpu, run_oracle, to_dev, tuning

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("inplace,width,split", [(0, 4, 0), (1, 4, 0), (0, 1, 0), (0, 4, 1), (1, 4, 1), (0, 1, 1)])
def test_batched_equals_plain_per_job(inplace, width, split):
    """Fused row pass (split = 0) and split update / gather passes (split =
    1), each FFT buffer option and column width."""
    from paper_2205_04295_amd import api, tune
    specs = [dict(seed=71, H=160, N=64, M=1, J=9), dict(seed=72, H=256, N=128, M=3, J=5),
             dict(seed=73, H=320, N=192, M=2, J=3), dict(seed=74, H=384, N=256, M=4, J=4),
             dict(seed=75, H=128, N=64, M=5, J=12)]
    ws = [wl.small_case(name=f"b{i}", **s) for i, s in enumerate(specs)]
    prm = dict(ws[0].params, iterations=2)
    devs = [to_dev(w) for w in ws]
    jobs = [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"],
                 err=torch.zeros(2, dtype=torch.float32, device="cuda:0"),
                 status=torch.zeros(1, dtype=torch.int32, device="cuda:0")) for d in devs]
    # the launch's tuning is that of its largest probe size, batch class
    saved = tune.get_tuning(256, True)
    try:
        tune.set_tuning(256, True, **dict(saved, rows_inplace=inplace, cols_width=width, rows_split=split))
        api.rpie_batched(jobs, **prm)
        torch.cuda.synchronize()
    finally:
        tune.set_tuning(256, True, **saved)
    for w, j in zip(ws, jobs):
        g = run_gpu(w, prm)
        assert rel_l2(j["obj"].cpu().numpy(), g["O"]) < 1e-5
        assert rel_l2(j["probe"].cpu().numpy(), g["P"]) < 1e-5
        assert np.allclose(j["err"].cpu().numpy(), g["err"], rtol=1e-5, atol=0)
        assert int(j["status"].item()) == 0
    o = run_oracle(ws[1], prm)
    assert rel_l2(jobs[1]["obj"].cpu().numpy(), o["O"]) < 1e-4
    assert rel_l2(jobs[1]["probe"].cpu().numpy(), o["P"]) < 1e-4


def test_batched_more_jobs_than_one_launch():
    """More jobs than one launch's job table holds (36), on each of the two
    streams: the driver deals each stream's share to 36 launch lanes, and
    the 4 jobs left over start when a lane frees up.  80 equal jobs of
    64^2 x 1 through the row / column passes (the default in batches) give
    bitwise equal results whichever stream, lane and start tick they get,
    and match the single-job sweep to float rounding; 40 through the
    one-workgroup LDS sweep (forced by the tuning) equal the single-job LDS
    sweep bitwise."""
    from paper_2205_04295_amd import api
    w = wl.small_case(81, 96, 64, 1, 4, name="many")
    prm = dict(w.params, iterations=1)
    ref = run_gpu(w, prm)            # single job: the LDS sweep
    devs = [to_dev(w) for _ in range(80)]
    jobs = [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"]) for d in devs]
    api.rpie_batched(jobs, **prm)
    torch.cuda.synchronize()
    first = jobs[0]["obj"].cpu().numpy()
    assert rel_l2(first, ref["O"]) < 1e-5
    for j in jobs:
        assert np.array_equal(j["obj"].cpu().numpy(), first)
    with tuning(64, 2, lds_sweep=1):
        devs = [to_dev(w) for _ in range(40)]
        jobs = [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"]) for d in devs]
        api.rpie_batched(jobs, **prm)
        torch.cuda.synchronize()
    for j in jobs:
        assert np.array_equal(j["obj"].cpu().numpy(), ref["O"])


def test_batched_many_jobs_in_place_passes():
    """18 jobs in one launch (the column pass then runs in place as well):
    each job's object and probe match its plain sweep to float rounding."""
    from paper_2205_04295_amd import api
    specs = [dict(seed=90 + i, H=192 if i % 2 else 256, N=128, M=1 + i % 3, J=3 + i % 4) for i in range(18)]
    ws = [wl.small_case(name=f"m{i}", **s) for i, s in enumerate(specs)]
    prm = dict(ws[0].params, iterations=2)
    devs = [to_dev(w) for w in ws]
    jobs = [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"]) for d in devs]
    api.rpie_batched(jobs, **prm)
    torch.cuda.synchronize()
    for w, j in zip(ws, jobs):
        g = run_gpu(w, prm)
        assert rel_l2(j["obj"].cpu().numpy(), g["O"]) < 1e-5
        assert rel_l2(j["probe"].cpu().numpy(), g["P"]) < 1e-5
    o = run_oracle(ws[4], prm)
    assert rel_l2(jobs[4]["obj"].cpu().numpy(), o["O"]) < 1e-4
    assert rel_l2(jobs[4]["probe"].cpu().numpy(), o["P"]) < 1e-4


def test_batched_large_probes_in_place_columns_many_modes():
    """16 jobs of 192^2 and 256^2 probes with 1, 3 and 5 modes (the column
    pass runs in place with its first and last stages in registers, for the
    widest mode capacity too): each job matches its plain sweep to float
    rounding, and the oracle to the plain sweep's tolerance."""
    from paper_2205_04295_amd import api
    specs = [dict(seed=110 + i, H=(192, 256)[i % 2] + 64, N=(192, 256)[i % 2], M=(1, 3, 5)[i % 3], J=3 + i % 3)
             for i in range(16)]
    ws = [wl.small_case(name=f"w{i}", **s) for i, s in enumerate(specs)]
    prm = dict(ws[0].params, iterations=2)
    devs = [to_dev(w) for w in ws]
    jobs = [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"],
                 err=torch.zeros(2, dtype=torch.float32, device="cuda:0")) for d in devs]
    api.rpie_batched(jobs, **prm)
    torch.cuda.synchronize()
    for w, j in zip(ws, jobs):
        g = run_gpu(w, prm)
        assert rel_l2(j["obj"].cpu().numpy(), g["O"]) < 1e-5
        assert rel_l2(j["probe"].cpu().numpy(), g["P"]) < 1e-5
        assert np.allclose(j["err"].cpu().numpy(), g["err"], rtol=1e-5, atol=0)
    o = run_oracle(ws[5], prm)  # 256^2 x 5 modes
    assert rel_l2(jobs[5]["obj"].cpu().numpy(), o["O"]) < 1e-4
    assert rel_l2(jobs[5]["probe"].cpu().numpy(), o["P"]) < 1e-4


def test_batched_calls_from_two_host_threads():
    """Two host threads issue batched calls on two streams at once (both fork
    the library's side stream): every job ends bitwise equal to the same call
    made alone."""
    import threading
    from paper_2205_04295_amd import api
    specs = [dict(seed=91, H=256, N=128, M=2, J=6), dict(seed=92, H=192, N=64, M=3, J=8),
             dict(seed=93, H=320, N=128, M=1, J=5)]
    ws = [wl.small_case(name=f"t{i}", **s) for i, s in enumerate(specs)]
    prm = dict(ws[0].params, iterations=2)

    def jobs():
        return [dict(obj=d["obj"], probe=d["probe"], pos=d["pos"], intens=d["I"]) for d in map(to_dev, ws)]
    ref = jobs()
    api.rpie_batched(ref, **prm)
    torch.cuda.synchronize()
    runs = [jobs(), jobs()]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()  # inputs uploaded on the default stream
    errors = []

    def work(k):
        try:
            with torch.cuda.stream(streams[k]):
                api.rpie_batched(runs[k], stream=streams[k], **prm)
        except Exception as e:  # surfaced below
            errors.append(e)
    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert not errors
    for run in runs:
        for a, b in zip(run, ref):
            assert torch.equal(a["obj"], b["obj"]) and torch.equal(a["probe"], b["probe"])
