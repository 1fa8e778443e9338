"""GPU parity of the direct recombination form (Taylor order 0: occupancies only): every
voxel against the FP64 oracle, against the levelled forms, and its default choice."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests.helpers import assert_parity, to_dsx

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


CASES = [  # (n, sites, configurations, closed box, hmax)
    ((12, 12, 12), 1, 1, False, 2),
    ((10, 7, 9), 2, 1, True, 1),
    ((6, 5, 8), 3, 3, True, 2),
    ((16, 16, 16), 1, 4, True, 1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_direct_form_matches_oracle_and_levelled_forms(case):
    import torch
    n, S, M, closed, hmax = CASES[case]
    frac = np.random.default_rng([61, case]).random((S, 3)) if S > 1 else None
    b = np.linspace(0.7, 1.3, S) if S > 1 else None
    m = synth.compositional(workload=60, model=case, n=n, M=M, hmax=hmax, closed=closed, frac=frac, b=b)
    say(f"direct form: n={n} S={S} M={M} box {m.count}")
    h = to_dsx(m)
    ref = O.intensity(m).reshape(m.count)
    outs = {}
    for v in (5, 2, 0):
        h.tune_set(v, 0, 12)
        o = torch.full(tuple(m.count), -1.0, device="cuda")
        h.compute_intensity(o)
        torch.cuda.synchronize()
        outs[v] = o.cpu().numpy()
        assert_parity(outs[v], ref, what=f"form {v}")
    # the default is the direct form for one or two sites x configurations
    if S * M <= 2:
        assert np.array_equal(outs[0], outs[5])
    h.close()


def test_direct_form_in_a_merged_batch():
    import torch
    import paper_1809_07088_amd as dsx
    models = [synth.compositional(workload=62, model=i, n=12 if i % 3 else 9, M=1, hmax=2) for i in range(48)]
    say("merged batch of direct-form models")
    hs = [to_dsx(mm) for mm in models]
    for h in hs:
        h.tune_set(5, 0, 12)
    outs = [torch.full(tuple(mm.count), -1.0, device="cuda") for mm in models]
    batch = dsx.Batch(hs, outs, mode=dsx.BATCH_MERGED)
    batch.run()
    torch.cuda.synchronize()
    for k in (0, 1, 2, 30, 47):
        alone = torch.empty(tuple(models[k].count), device="cuda")
        hs[k].compute_intensity(alone)
        torch.cuda.synchronize()
        assert torch.equal(alone, outs[k]), k
        assert_parity(outs[k].cpu().numpy(), O.intensity(models[k]).reshape(models[k].count))
    batch.close()
    for h in hs:
        h.close()


def test_direct_form_rejected_where_it_does_not_apply():
    import paper_1809_07088_amd as dsx
    m = synth.displacive(workload=63, n=8, M=1, order=2, hmax=1)
    say("direct form on an order-2 model")
    h = to_dsx(m)
    with pytest.raises(dsx.DsxError) as e:
        h.tune_set(5, 0, 12)
    assert e.value.status == dsx.ERR_ARG
    h.close()


def test_direct_form_filtered_on_half_stored_box():
    """The filter's grown box of a symmetric output box is stored as its planes G1 <= 0:
    the direct form computes exactly those (the filtered output matches the oracle and
    the levelled form), and two models served side by side keep each other's results."""
    import torch
    import paper_1809_07088_amd as dsx
    m = synth.compositional(workload=64, model=0, n=(8, 7, 9), M=1, hmax=1, closed=True)
    say(f"direct form, filtered, symmetric box {m.count}")
    h = to_dsx(m)
    ref = O.filtered_intensity(m, 2, 1)
    outs = {}
    for v in (5, 2):
        h.tune_set(v, 0, 12)
        o = torch.full(tuple(m.count), -1.0, device="cuda")
        h.noise_filter(2, 1, o)
        torch.cuda.synchronize()
        outs[v] = o.cpu().numpy()
        assert_parity(outs[v], ref, what=f"form {v}")
    h.close()
    # adjacent workspaces in one server arena: a round of both models, filtered
    other = synth.displacive(workload=64, model=1, n=8, M=1, order=3, hmax=1)
    srv = dsx.Server(slots=1, queue_capacity=16, arena_bytes=1 << 30, max_round=16)
    from tests.test_gpu_serving import served
    hs = [served(srv, mm) for mm in (m, other)]
    for _ in range(3):
        o = [torch.full(tuple(mm.count), -1.0, device="cuda") for mm in (m, other)]
        ts = [srv.submit(hh, oo, lanczos_m=2) for hh, oo in zip(hs, o)]
        for t in ts:
            assert srv.wait(t, 60000)
        assert_parity(o[0].cpu().numpy(), ref)
        assert_parity(o[1].cpu().numpy(), O.filtered_intensity(other, 2, 1))
    srv.close()
