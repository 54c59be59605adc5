"""GPU tests of the job server (srv_*): jobs that run side by side give the
same bits as the oracle and as the same job run alone; admission keeps the
projected footprints of running jobs within the budget; failures stay with
their job.  Each case prints its name before it touches the GPU."""
import sys

import numpy as np
import pytest

import oracle
import qcircuits as qc

pytestmark = pytest.mark.gpu

cq = pytest.importorskip("paper_1811_05630_amd")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


GROVER, QFT, LAYERED = 0, 1, 2


def mix():
    """Small jobs of the three families, both precisions, several bounds."""
    jobs = []
    n = 10
    jobs.append(dict(n=n, sl=7, eb=1e-6, gates=qc.grover(n, 613, 2), family=GROVER, fp32=False))
    n = 11
    jobs.append(dict(n=n, sl=8, eb=1e-5, gates=qc.qft(n), family=QFT, fp32=True, init=("basis", 1234)))
    n = 9
    jobs.append(dict(n=n, sl=6, eb=3e-6, gates=qc.random_layered(n, 3, seed=5), family=LAYERED, fp32=False))
    n = 12
    jobs.append(dict(n=n, sl=9, eb=1e-4, gates=qc.grover(n, 77, 1), family=GROVER, fp32=True))
    n = 10
    th, ph = qc.product_angles(n, 3)
    jobs.append(dict(n=n, sl=8, eb=2e-6, gates=qc.qft(n), family=QFT, fp32=False,
                     init=("product", qc.product_factors(th, ph))))
    n = 8
    jobs.append(dict(n=n, sl=5, eb=1e-7, gates=qc.random_layered(n, 2, seed=9), family=LAYERED, fp32=True))
    return jobs


def submit(srv, j, **extra):
    init = j.get("init")
    kw = dict(family=j["family"], fp32=j["fp32"], chunk_log2=5, out_count=1 << j["n"], **extra)
    if init is not None:
        kw["init"] = init[0]
        if init[0] == "basis":
            kw["basis"] = init[1]
        else:
            kw["factors"] = init[1]
    return srv.submit(j["n"], j["sl"], j["eb"], cq.Circuit(j["gates"]), **kw)


def run_oracle(j):
    o = oracle.OracleSim(j["n"], j["sl"], 5, j["eb"], oracle.ABS | (oracle.FP32 if j["fp32"] else 0))
    init = j.get("init")
    if init is not None:
        (o.init_basis if init[0] == "basis" else o.init_product)(init[1])
    o.apply(j["gates"])
    return o


def run_alone(j):
    s = cq.Sim(j["n"], j["sl"], j["eb"], chunk_log2=5, fp32=j["fp32"])
    init = j.get("init")
    if init is not None:
        (s.init_basis if init[0] == "basis" else s.init_product)(init[1])
    s.apply(j["gates"])
    return s


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def test_mixed_jobs_match_the_oracle_and_running_alone():
    jobs = mix()
    say("serve: 6 mixed jobs, 3 at a time")
    with cq.Server(budget_bytes=8 << 30, max_active=3) as srv:
        ids = [submit(srv, j) for j in jobs]
        done = {d["id"]: d for d in srv.drain(timeout=300)}
    assert sorted(done) == sorted(ids)
    starts = sorted((d["t_start"], d["t_end"]) for d in done.values())
    overlapped = any(starts[i + 1][0] < starts[i][1] for i in range(len(starts) - 1))
    for i, j in zip(ids, jobs):
        d = done[i]
        assert d["status"] == 0, d["error"]
        assert d["applied"] == len(j["gates"])
        o = run_oracle(j)
        assert np.array_equal(bits(d["amplitudes"]), bits(o.amplitudes())), f"job {i} vs oracle"
        assert d["stats"]["compressed_bytes"] == o.total_bytes()
        say(f"serve: job {i} alone")
        s = run_alone(j)
        st = s.stats()
        assert np.array_equal(bits(d["amplitudes"]), bits(s.amplitudes())), f"job {i} mixed vs alone"
        for k in ("compressed_bytes", "peak_compressed", "escapes", "passes", "max_abs_codec_err"):
            assert d["stats"][k] == st[k], (i, k)
        s.close()
    # the six jobs were queued together and three workers run them: their
    # service intervals must overlap (continuous batching, not a queue)
    assert overlapped, f"no two jobs ran at the same time: {starts}"


def test_admission_keeps_running_footprints_within_the_budget():
    n, sl, eb = 12, 9, 1e-6
    gates = cq.Circuit(qc.qft(n))
    say("serve: admission with room for two jobs")
    with cq.Server(budget_bytes=1 << 40, max_active=4) as probe:
        one = probe.projected_bytes(n, sl, eb, family=QFT, chunk_log2=5)
    budget = int(2.5 * one)
    with cq.Server(budget_bytes=budget, max_active=4) as srv:
        ids = [srv.submit(n, sl, eb, gates, family=QFT, chunk_log2=5, init="basis", basis=5 + k)
               for k in range(6)]
        done = srv.drain(timeout=300)
    assert sorted(d["id"] for d in done) == ids
    for d in done:
        assert d["status"] == 0, d["error"]
        assert d["projected_bytes"] <= one  # the model only lowers a family's projection
    ev = sorted([(d["t_start"], d["projected_bytes"]) for d in done] +
                [(d["t_end"], -d["projected_bytes"]) for d in done], key=lambda e: (e[0], e[1]))
    load = peak = 0
    for _, b in ev:
        load += b
        peak = max(peak, load)
    assert peak <= budget


def test_footprint_is_what_a_new_handle_holds():
    for n, sl, kw in [(10, 7, {}), (12, 9, dict(fp32=True)), (14, 10, dict(arena_bytes=1 << 20)),
                      (11, 11, dict(workspace_bytes=1 << 20))]:
        say(f"footprint n={n} sl={sl} {kw}")
        s = cq.Sim(n, sl, 1e-6, use_torch=False, **kw)
        assert s.stats()["device_bytes"] == cq.footprint(n, sl, 1e-6, **kw)
        s.close()


def test_ratio_model_learns_from_finished_jobs():
    n, sl, eb = 16, 12, 1e-5  # large enough that arenas are above their 64 KiB floor
    gates = cq.Circuit(qc.grover(n, 99, 1))
    say("serve: ratio model")
    with cq.Server(budget_bytes=8 << 30, max_active=2) as srv:
        before = srv.projected_bytes(n, sl, eb, family=GROVER)
        other = srv.projected_bytes(n, sl, eb, family=QFT)
        assert before == other
        srv.submit(n, sl, eb, gates, family=GROVER)
        (d,) = srv.drain(timeout=120)
        assert d["status"] == 0, d["error"]
        after = srv.projected_bytes(n, sl, eb, family=GROVER)
        assert after < before
        assert srv.projected_bytes(n, sl, eb, family=QFT) == other
        r = d["stats"]["min_ratio"]
        arena = max(min(8 << n, int(1.25 * (16 << n) / r)), 64 << 10)
        assert after == cq.footprint(n, sl, eb, arena_bytes=arena)


def test_a_failing_job_does_not_disturb_the_others():
    n, sl, eb = 10, 7, 1e-6
    bad = qc.H(n + 3)  # target outside the register
    say("serve: one bad job among good ones")
    with cq.Server(budget_bytes=8 << 30, max_active=3) as srv:
        good = [srv.submit(n, sl, eb, cq.Circuit(qc.qft(n)), family=QFT, init="basis", basis=k, out_count=16)
                for k in range(3)]
        wrong = srv.submit(n, sl, eb, [qc.H(0), bad], family=QFT)
        done = {d["id"]: d for d in srv.drain(timeout=120)}
        with pytest.raises(cq.SimError) as e:
            srv.submit(40, 20, eb, family=QFT)  # projected far above the budget
        assert e.value.rc == -2
        with pytest.raises(cq.SimError) as e:
            srv.submit(n, sl, eb, family=cq.SRV_FAMILIES)
        assert e.value.rc == -1
    assert done[wrong]["status"] == -1 and "target" in done[wrong]["error"]
    ref = run_alone(dict(n=n, sl=sl, eb=eb, gates=qc.qft(n), fp32=False, init=("basis", 0)))
    ampl = ref.amplitudes(0, 16)
    assert np.array_equal(bits(done[good[0]]["amplitudes"]), bits(ampl))
    for g in good:
        assert done[g]["status"] == 0


def test_server_runs_fused_relative_and_record_mode_jobs():
    """Jobs of other configurations (fused blocks, a relative bound, zero and
    constant chunks) on the server: the same bits as each one run alone."""
    jobs = [
        dict(n=10, sl=7, eb=1e-4, gates=qc.qft(10), kw=dict(relative=True), init=("basis", 9)),
        dict(n=11, sl=8, eb=1e-6, gates=qc.qft(11), kw=dict(fused=True), init=("basis", 5)),
        dict(n=12, sl=9, eb=1e-6, gates=qc.grover(12, 7, 1), kw=dict(zero_chunks=True, const_chunks=True)),
    ]
    say("serve: fused, relative and record-mode jobs")
    with cq.Server(budget_bytes=8 << 30, max_active=3) as srv:
        ids = []
        for j in jobs:
            kw = dict(j["kw"], chunk_log2=5, out_count=1 << j["n"], family=QFT)
            if "init" in j:
                kw.update(init="basis", basis=j["init"][1])
            ids.append(srv.submit(j["n"], j["sl"], j["eb"], cq.Circuit(j["gates"]), **kw))
        done = {d["id"]: d for d in srv.drain(timeout=300)}
    for i, j in zip(ids, jobs):
        d = done[i]
        assert d["status"] == 0, d["error"]
        s = cq.Sim(j["n"], j["sl"], j["eb"], chunk_log2=5, **j["kw"])
        if "init" in j:
            s.init_basis(j["init"][1])
        s.apply(j["gates"])
        assert np.array_equal(bits(d["amplitudes"]), bits(s.amplitudes())), f"job {i}"
        assert d["stats"]["compressed_bytes"] == s.stats()["compressed_bytes"]
        s.close()
