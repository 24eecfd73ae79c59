"""Batched persistent execution, graph replay and the autotuner (needs an MI355X).

Every output is compared byte for byte with the source text and with the
CPU oracle's two-pass result on the same seeded input.
"""
import time

import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gz():
    import paper_1905_07224_amd as gz
    return gz


def _dev(b):
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def files():
    # C1-like files of several sizes and levels (seeded)
    out = []
    for k, (size, level) in enumerate([(1 << 20, 6), (3 << 20, 1), (600 << 10, 9), (2 << 20, 6), (64 << 10, 6)]):
        raw = synth.fastq_like(size, 40 + k)
        out.append((raw, synth.gzip_member(raw, level)))
    return out


def _outs(files):
    return [torch.zeros(len(r) + 64, dtype=torch.uint8, device="cuda:0") for r, _ in files]


def test_batch_matches_oracle(orc, files):
    gz = _gz()
    _say("batch of", len(files), "files, eager")
    outs = _outs(files)
    bp = gz.BatchPlan([_dev(c) for _, c in files], [4, 8, 3, 5, 1], outs=outs)
    bp.launch()
    for i, (raw, comp) in enumerate(files):
        r = bp.result(i)
        assert r.status == 0 and r.out_len == len(raw)
        got = outs[i][: r.out_len].cpu().numpy().tobytes()
        ref = orc.pugz(comp, [4, 8, 3, 5, 1][i])
        assert ref.status == orc.OK
        assert got == raw == ref.out.tobytes()


def test_graph_replays_equal_eager(files):
    """The captured pass sequence replayed several times, with eager work and
    synchronisations between replays; every replay equals the eager run."""
    gz = _gz()
    _say("batch graph replays")
    outs = _outs(files)
    bp = gz.BatchPlan([_dev(c) for _, c in files], [4, 8, 3, 5, 1], outs=outs)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bp.launch(s)
    s.synchronize()
    eager = [o.clone() for o in outs]
    stats = [bp.result(i).as_dict() for i in range(len(files))]
    for rep in range(4):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        scratch = torch.randn(1 << 20, device="cuda:0").sum().item()  # eager work between replays
        assert scratch == scratch
        bp.launch_graph(s)
        s.synchronize()
        for i, (raw, _) in enumerate(files):
            r = bp.result(i)
            assert r.as_dict() == stats[i], (rep, i)
            assert torch.equal(outs[i], eager[i]), (rep, i)
            assert outs[i][: r.out_len].cpu().numpy().tobytes() == raw


def test_graph_single_file(files):
    gz = _gz()
    _say("one-file graph")
    raw, comp = files[1]
    plan = gz.Plan(_dev(comp), 6)
    out = torch.zeros(len(raw) + 16, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        plan.launch_graph(out, s)
        s.synchronize()
        r = plan.result()
        assert r.status == 0 and out[: r.out_len].cpu().numpy().tobytes() == raw, rep


def test_graph_rejects_null_stream_and_timing(files):
    gz = _gz()
    raw, comp = files[0]
    plan = gz.Plan(_dev(comp), 2, timing=1)
    ws = plan.workspace()
    import ctypes as C
    assert gz.lib().gz_decompress_graph(plan._h, C.c_void_p(ws.data_ptr()), ws.numel(), None) == gz.GZ_E_ARG
    s = torch.cuda.Stream()
    assert gz.lib().gz_decompress_graph(plan._h, C.c_void_p(ws.data_ptr()), ws.numel(),
                                        C.c_void_p(s.cuda_stream)) == gz.GZ_E_ARG


def test_autotune_choice_is_exact_and_cached(orc, files):
    import time

    gz = _gz()
    _say("autotune")
    raw, comp = files[1]
    d = _dev(comp)
    t0 = time.perf_counter()
    best = gz.autotune(d)
    t1 = time.perf_counter()
    again = gz.autotune(d)
    t2 = time.perf_counter()
    assert best == again
    assert best["chunk_bytes"] in (32 << 10, 40 << 10, 64 << 10, 128 << 10, 256 << 10, 1 << 20)
    assert best["window_syms"] in (512, 1024, 2048)
    assert t2 - t1 < t1 - t0  # the second answer comes from the cache
    out = gz.decompress(d, 0, **best)
    assert out.cpu().numpy().tobytes() == raw


def test_tuned_option_in_batch_and_server(orc, files):
    """opts.tuned: once gz_autotune has timed a file's class, a batch plans
    that class's files with the tuned chunk size (files of other classes keep
    the default), the serving loop too, and the outputs stay the oracle's."""
    gz = _gz()
    _say("tuned batch")
    comps = [_dev(c) for _, c in files]
    best = gz.autotune(comps[1])
    want = sum(gz.Plan(c, 0, **(best if k == 1 else {})).n_chunks for k, c in enumerate(comps))
    outs = _outs(files)
    bp = gz.BatchPlan(comps, 0, outs=outs, tuned=1)
    assert bp.info.n_chunks == want
    bp.launch()
    for k, (raw, comp) in enumerate(files):
        r = bp.result(k)
        assert r.status == 0 and outs[k][:r.out_len].cpu().numpy().tobytes() == raw
    if best["chunk_bytes"] != gz.DEFAULT_CHUNK_BYTES:
        assert gz.BatchPlan(comps, 0, outs=outs).info.n_chunks != want
    srv = gz.Server(budget_bytes=8 << 30, max_inflight=2, max_batch=4, tuned=1)
    outs = _outs(files)
    for k, c in enumerate(comps):
        srv.submit(c, outs[k], k)
    done = {}
    for _ in range(20000):
        for d in srv.poll():
            done[d["tag"]] = d
        if len(done) == len(files):
            break
        time.sleep(0.001)
    srv.close()
    assert sorted(done) == list(range(len(files)))
    for k, (raw, _) in enumerate(files):
        assert done[k]["status"] == 0 and outs[k][:len(raw)].cpu().numpy().tobytes() == raw


def test_serving_mix_equals_alone(files):
    """Jobs through the serving loop, with a budget that forces queueing, give
    the bytes each job gives alone; the arena never exceeds the budget."""
    import time

    gz = _gz()
    _say("serving loop, mixed jobs")
    comps = [_dev(c) for _, c in files]
    alone = [gz.decompress(c, 0).cpu().numpy().tobytes() for c in comps]
    biggest = max(gz.Plan(c, 0).info.ws_bytes for c in comps)
    budget = int(biggest * 2.5)
    srv = gz.Server(budget_bytes=budget, max_inflight=3, max_batch=4)
    outs, want = {}, {}
    order = [0, 1, 2, 3, 4, 1, 0, 3, 2, 4, 1, 1]
    for tag, k in enumerate(order):
        outs[tag] = torch.zeros(len(files[k][0]) + 32, dtype=torch.uint8, device="cuda:0")
        want[tag] = k
        srv.submit(comps[k], outs[tag], tag)
    done = []
    t0 = time.time()
    while len(done) < len(order) and time.time() - t0 < 60:
        done += srv.poll()
        time.sleep(0.0005)
    st = srv.stats()
    srv.close()
    assert len(done) == len(order)
    for d in done:
        k = want[d["tag"]]
        assert d["status"] == 0 and d["out_len"] == len(files[k][0])
        got = outs[d["tag"]][: d["out_len"]].cpu().numpy().tobytes()
        assert got == alone[k] == files[k][0]
        assert d["t_submit"] <= d["t_start"] <= d["t_end"]
    assert st["arena_peak"] <= budget and st["batches"] >= 2
    assert st["resident_peak"] <= budget


def test_serving_admits_while_batches_run(files):
    """Continuous batching: jobs submitted while earlier batches are still on
    the GPU are admitted into batches that run beside them (a job starts
    before a job admitted earlier has finished), and each result equals the
    job decoded alone."""
    import time

    gz = _gz()
    _say("serving loop, arrivals during running batches")
    comps = [_dev(c) for _, c in files]
    alone = [gz.decompress(c, 0).cpu().numpy().tobytes() for c in comps]
    srv = gz.Server(budget_bytes=8 << 30, max_inflight=4, max_batch=2)
    outs, want, running_at_submit = {}, {}, []
    order = [4, 3, 4, 3, 2, 1, 0, 4, 3, 2, 1, 0]
    done = []
    t0 = time.time()
    for tag, k in enumerate(order):
        outs[tag] = torch.zeros(len(files[k][0]) + 32, dtype=torch.uint8, device="cuda:0")
        want[tag] = k
        if tag >= 2:
            # later jobs arrive while what was admitted before is on the GPU
            while srv.stats()["running"] == 0 and time.time() - t0 < 30:
                done += srv.poll()
            running_at_submit.append(srv.stats()["running"])
        srv.submit(comps[k], outs[tag], tag)
        done += srv.poll()
    while len(done) < len(order) and time.time() - t0 < 60:
        done += srv.poll()
        time.sleep(0.0002)
    srv.close()
    assert len(done) == len(order)
    for d in done:
        k = want[d["tag"]]
        assert d["status"] == 0
        assert outs[d["tag"]][: d["out_len"]].cpu().numpy().tobytes() == alone[k] == files[k][0]
    assert all(r > 0 for r in running_at_submit)
    by = {d["tag"]: d for d in done}
    overlap = [(a, b) for a in by for b in by if b > a and by[b]["t_submit"] > by[a]["t_start"]
               and by[b]["t_start"] < by[a]["t_end"]]
    assert overlap, "no job was admitted while an earlier one ran"
