"""GPU tests of the serving loop: every request computed in a mix of concurrent
requests equals, bit for bit, the same request computed alone, and matches the
FP64 oracle; admission by workspace size and queue capacity."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests.helpers import edge_sample_indices, oracle_filtered_at, assert_parity, max_rel, MAXTOL, desc_kwargs, rel_l2, to_dsx

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def variant_sites(model, seed):
    """New variables for configuration 0 of `model` (same kind and shape), seeded."""
    r = np.random.default_rng([5, 77, seed])
    S, nn = model.n_sites, tuple(model.n)
    occ = disp = spin = None
    if model.occ is not None:
        occ = (r.random((S,) + nn) < 0.5).astype(np.float32)
    if model.disp is not None:
        disp = synth.correlated_displacements(r, 1, S, nn)[0]
    if model.spin is not None:
        v = r.normal(size=(S,) + nn + (3,))
        spin = (v / np.linalg.norm(v, axis=-1, keepdims=True)).astype(np.float32)
    return occ, disp, spin


def with_sites(model, sites):
    import copy
    m = copy.copy(model)
    occ, disp, spin = sites
    m.occ = None if occ is None else occ[None]
    m.disp = None if disp is None else disp[None]
    m.spin = None if spin is None else spin[None]
    return m


def served(server, model):
    import torch
    h = server.add_model(**desc_kwargs(model))
    h.set_grid(model.g0, model.count)
    for c in range(model.n_configs):
        h.set_sites(c, *[None if a is None else torch.from_numpy(np.ascontiguousarray(a[c])).cuda()
                         for a in (model.occ, model.disp, model.spin)])
    return h


def dev(sites):
    import torch
    return [None if a is None else torch.from_numpy(a).cuda() for a in sites]


MIX = [(0, 8, 3, 0), (1, 8, 2, 1), (2, 8, 4, 2), (3, 12, 6, 1), (4, 16, 5, 0), (5, 10, 16, 2),
       (6, 20, 3, 1)]


def test_alone_equals_mix_and_oracle():
    import torch
    import paper_1809_07088_amd as dsx
    models = [synth.serving_request_model(workload=50, model=i, n=n, S=S, typ=t, order=5)
              for (i, n, S, t) in MIX]
    srv = dsx.Server(slots=4, queue_capacity=256, arena_bytes=2 << 30)
    hs = [served(srv, m) for m in models]
    variants = {(i, v): dev(variant_sites(m, 10 * i + v)) for i, m in enumerate(models) for v in range(2)}
    jobs = [(i, v, lm) for i in range(len(models)) for v in range(2) for lm in (0, 2)]

    def out_for(i, lm):      # oversample 1: the filtered output has the box's shape too
        return torch.full(tuple(models[i].count), -7.0, device="cuda")

    say(f"serving alone: {len(jobs)} requests one at a time")
    alone = {}
    for (i, v, lm) in jobs:
        o = out_for(i, lm)
        t = srv.submit(hs[i], o, 0, *variants[(i, v)], lanczos_m=lm)
        assert srv.wait(t, 60000)
        alone[(i, v, lm)] = o.cpu()
    say("serving the same requests as one burst, shuffled")
    order = np.random.default_rng(3).permutation(len(jobs))
    outs, tickets = {}, []
    for k in order:
        i, v, lm = jobs[k]
        outs[jobs[k]] = out_for(i, lm)
        tickets.append(srv.submit(hs[i], outs[jobs[k]], 0, *variants[(i, v)], lanczos_m=lm))
    for t in tickets:
        assert srv.wait(t, 60000)
    st = srv.stats()
    assert st["completed"] == 2 * len(jobs) and st["failed"] == 0
    assert st["peak_in_flight"] >= 2          # requests overlapped on the device
    for key, o in outs.items():
        assert torch.equal(o.cpu(), alone[key]), key
    # the direct (non-served) path computes the same bits
    i, v = 3, 1
    plain = to_dsx(with_sites(models[i], [a for a in variant_sites(models[i], 10 * i + v)]))
    ref = torch.empty(tuple(models[i].count), device="cuda")
    plain.compute_intensity(ref)
    torch.cuda.synchronize()
    assert torch.equal(ref.cpu(), alone[(i, v, 0)])
    plain.close()
    # FP64 oracle: whole boxes of the small models, sampled voxels of the larger ones
    for (i, v, lm) in jobs:
        m = with_sites(models[i], variant_sites(models[i], 10 * i + v))
        got = alone[(i, v, lm)].numpy()
        if m.n[0] <= 8:
            exp = O.filtered_intensity(m, lm, 1) if lm else O.intensity(m).reshape(m.count)
            assert_parity(got, exp, what=str((i, v, lm)))
            continue
        idx = edge_sample_indices(m.count, 128, 7 * i + v)
        Q = idx + np.asarray(m.g0)
        exp = oracle_filtered_at(m, Q, lm) if lm else O.intensity(m, Q.astype(np.int32))
        assert_parity(got[tuple(idx.T)], exp, what=str((i, v, lm)))
    srv.close()


def test_same_model_requests_keep_submission_order():
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.serving_request_model(workload=51, model=0, n=12, S=4, typ=1, order=4)
    srv = dsx.Server(slots=4, queue_capacity=64, arena_bytes=1 << 30)
    h = served(srv, m)
    say("same-model requests in a burst")
    vs = [variant_sites(m, 100 + k) for k in range(6)]
    outs = [torch.empty(tuple(m.count), device="cuda") for _ in vs]
    ts = [srv.submit(h, o, 0, *dev(v)) for o, v in zip(outs, vs)]
    for t in ts:
        assert srv.wait(t, 60000)
    for o, v in zip(outs, vs):
        plain = to_dsx(with_sites(m, v))
        ref = torch.empty(tuple(m.count), device="cuda")
        plain.compute_intensity(ref)
        torch.cuda.synchronize()
        assert torch.equal(o.cpu(), ref.cpu())
        plain.close()
    srv.close()


def test_admission_by_workspace_and_queue_capacity():
    import torch
    import paper_1809_07088_amd as dsx
    big = synth.serving_request_model(workload=52, model=0, n=32, S=8, typ=1, order=6)
    info = dsx.plan_query(**desc_kwargs(big))
    ws = int(info.spectrum_bytes) + (1 << 24)
    # an arena that holds one such request at a time: requests run one by one
    srv = dsx.Server(slots=4, queue_capacity=1, arena_bytes=ws + ws // 2)
    h = served(srv, big)
    say("admission: arena for one request, queue of one")
    sites = [dev(variant_sites(big, 200 + k)) for k in range(12)]
    bufs = [torch.empty(tuple(big.count), device="cuda") for _ in range(12)]
    torch.cuda.synchronize()
    outs, ts, busy = [], [], 0
    for o, v in zip(bufs, sites):     # a tight burst: the queue of one overflows
        try:
            ts.append(srv.submit(h, o, 0, *v))
            outs.append(o)
        except dsx.DsxError as e:
            assert e.status == dsx.ERR_BUSY
            busy += 1
    for t in ts:
        assert srv.wait(t, 60000)
    st = srv.stats()
    assert busy >= 1 and st["rejected"] == busy
    assert st["peak_in_flight"] == 1 and st["arena_peak_bytes"] <= st["arena_bytes"]
    assert all(torch.isfinite(o).all() for o in outs)
    srv.close()
    # a request larger than the whole arena is refused at submission
    srv = dsx.Server(slots=2, queue_capacity=8, arena_bytes=1 << 20)
    h = served(srv, big)
    with pytest.raises(dsx.DsxError) as e:
        srv.submit(h, torch.empty(tuple(big.count), device="cuda"))
    assert e.value.status == dsx.ERR_NOMEM
    srv.close()


def test_served_model_rules():
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.serving_request_model(workload=53, model=0, n=8, S=2, typ=0)
    srv = dsx.Server(slots=1, queue_capacity=4, arena_bytes=64 << 20)
    say("served model rules")
    h = srv.add_model(**desc_kwargs(m))
    out = torch.empty(tuple(m.count), device="cuda")
    with pytest.raises(dsx.DsxError) as e:
        srv.submit(h, out, 0, *dev(variant_sites(m, 1)))
    assert e.value.status == dsx.ERR_STATE          # no grid yet
    h.set_grid(m.g0, m.count)
    with pytest.raises(dsx.DsxError) as e:
        h.compute_intensity(out)
    assert e.value.status == dsx.ERR_STATE          # served models compute through the server
    with pytest.raises(dsx.DsxError) as e:
        dsx.destroy_model(h.handle)
    assert e.value.status == dsx.ERR_ARG
    t = srv.submit(h, out)                           # sites of config 0 never set
    with pytest.raises(dsx.DsxError) as e:
        srv.wait(t, 60000)
    assert e.value.status == dsx.ERR_STATE
    t = srv.submit(h, out, 0, *dev(variant_sites(m, 2)))
    assert srv.wait(t, 60000)
    with pytest.raises(dsx.DsxError) as e:
        srv.wait(t, 0)                               # retired
    assert e.value.status == dsx.ERR_ARG
    st = srv.stats(reset=True)
    assert st["completed"] == 1 and st["failed"] == 1
    srv.close()


def test_merged_rounds_equal_single_requests():
    """A burst on a server that merges up to 16 requests per round gives, bit for bit, what
    a server running one request per slot gives, and forms rounds of several requests."""
    import torch
    import paper_1809_07088_amd as dsx
    models = [synth.serving_request_model(workload=54, model=i, n=n, S=S, typ=t, order=4)
              for i, (n, S, t) in enumerate([(8, 2, 0), (8, 3, 1), (10, 2, 2), (12, 4, 1), (9, 1, 0), (8, 5, 2),
                                             (11, 3, 1), (8, 1, 0)])]
    jobs = [(i, v, lm) for i in range(len(models)) for v in range(2) for lm in (0, 2)]
    variants = {(i, v): dev(variant_sites(m, 300 + 10 * i + v)) for i, m in enumerate(models) for v in range(2)}
    res = {}
    for mr in (1, 16):
        say(f"burst on a server with max_round={mr}")
        srv = dsx.Server(slots=2, queue_capacity=256, arena_bytes=2 << 30, max_round=mr)
        hs = [served(srv, m) for m in models]
        outs = {k: torch.full(tuple(models[k[0]].count), -3.0, device="cuda") for k in jobs}
        srv.stats(reset=True)
        ts = [srv.submit(hs[i], outs[(i, v, lm)], 0, *variants[(i, v)], lanczos_m=lm) for (i, v, lm) in jobs]
        for t in ts:
            assert srv.wait(t, 60000)
        st = srv.stats()
        assert st["completed"] == len(jobs) and st["failed"] == 0
        if mr == 1:
            assert st["round_requests"] == st["rounds"]
        else:
            assert st["round_requests"] > st["rounds"]       # some rounds held several requests
        res[mr] = {k: o.cpu() for k, o in outs.items()}
        srv.close()
    for k in jobs:
        assert torch.equal(res[1][k], res[16][k]), k
    i, v, lm = jobs[5]
    m = with_sites(models[i], variant_sites(models[i], 300 + 10 * i + v))
    exp = O.filtered_intensity(m, lm, 1) if lm else O.intensity(m).reshape(m.count)
    assert_parity(res[16][(i, v, lm)].numpy(), exp)
