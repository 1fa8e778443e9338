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
