"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and its
host-only planner counts fields and validates descriptions (no GPU calls)."""
import os
import re

import numpy as np
import pytest

import paper_1809_07088_amd as dsx
import synth
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "dsx.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:dsx_status|const char\*|int32_t)\s+(dsx_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = dsx.lib()
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(dsx.EXPORTS)
    assert dsx.version() >= 100


def golden(key):
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.txt")) as f:
        for line in f:
            if line.split() and line.split()[0] == key:
                return float(line.split()[1])
    raise KeyError(key)


def test_field_counts_match_paper():
    fcc = dict(cell=[1, 1, 1, 90, 90, 90], n=(8, 8, 8), frac=synth.FCC_BASIS, b=synth.FCC_B)
    info = dsx.plan_query(**fcc, taylor_order=5)
    assert info.fields_per_site == golden("ffts_fifth_order_total")        # 55
    assert dsx.plan_query(**fcc, taylor_order=5, has_occ=True).fields_per_site == 56
    for n in range(0, 9):
        full = dsx.plan_query(**fcc, taylor_order=n, has_occ=True).fields_per_site
        assert full == (n + 1) * (n + 2) * (n + 3) // 6
    for n in (12, 16):          # C(N+3, 3) fields up to the largest order
        assert dsx.plan_query(**fcc, taylor_order=n, has_occ=True).fields_per_site == (n + 1) * (n + 2) * (n + 3) // 6
    info = dsx.plan_query(**fcc, taylor_order=8, n_configs=3)
    assert info.fields_per_site == 164 and info.total_fields == 3 * 4 * 164
    assert info.n_classes == 2                       # r_mu3 in {0, 1/2}
    assert info.spectrum_bytes == 3 * 8 * 8 * 4 * 164 * 5 * 8


def test_magnetic_plan_and_classes():
    pyro = synth.pyrochlore_sites()
    info = dsx.plan_query(cell=[10, 10, 10, 90, 90, 90], n=(24, 24, 24), frac=pyro, b=np.ones(16),
                          kind=dsx.MAGNETIC, ff=np.tile(synth.MAG_FF, (16, 1)))
    assert info.fields_per_site == 3
    assert info.n_classes == 4                       # r_mu3 in {0, 1/4, 1/2, 3/4}
    # displacements of a magnetic model only feed its Debye-Waller factor (Eq. dw): still
    # three transforms per site, plus the resident displacements and their lattice sums
    dw = dsx.plan_query(cell=[10, 10, 10, 90, 90, 90], n=(24, 24, 24), frac=pyro, b=np.ones(16),
                        kind=dsx.MAGNETIC, ff=np.tile(synth.MAG_FF, (16, 1)), taylor_order=4)
    assert dw.fields_per_site == 3 and dw.spectrum_bytes == info.spectrum_bytes
    assert dw.device_bytes >= info.device_bytes + 16 * 24 ** 3 * 12


@pytest.mark.parametrize("kw,status", [
    (dict(n=(0, 4, 4)), dsx.ERR_ARG),
    (dict(n=(4, 4, 257)), dsx.ERR_UNSUPPORTED),
    (dict(taylor_order=17), dsx.ERR_UNSUPPORTED),
    (dict(taylor_order=-1), dsx.ERR_ARG),
    (dict(n_configs=0), dsx.ERR_ARG),
    (dict(cell=[1, 1, 1, 90, 90, 200]), dsx.ERR_ARG),
    (dict(cell=[0, 1, 1, 90, 90, 90]), dsx.ERR_ARG),
    (dict(kind=7), dsx.ERR_ARG),
    (dict(taylor_order=0, has_occ=False), dsx.ERR_ARG),
    (dict(norm_N=-1.0), dsx.ERR_ARG),
])
def test_plan_query_rejects_bad_descriptions(kw, status):
    base = dict(cell=[1, 1, 1, 90, 90, 90], n=(4, 4, 4), frac=[[0, 0, 0]], b=[1.0], taylor_order=2)
    base.update(kw)
    with pytest.raises(dsx.DsxError) as e:
        dsx.plan_query(**base)
    assert e.value.status == status
    assert dsx.last_error() != ""


def test_too_many_sites_unsupported():
    with pytest.raises(dsx.DsxError) as e:
        dsx.plan_query(cell=[1, 1, 1, 90, 90, 90], n=(4, 4, 4), frac=np.zeros((65, 3)), b=np.ones(65),
                       taylor_order=1)
    assert e.value.status == dsx.ERR_UNSUPPORTED


def _header_structs():
    """Field names, in order, of every `typedef struct { ... } name;` in include/dsx.h."""
    import re
    text = open(os.path.join(ROOT, "include", "dsx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"^(const\s+)?[\w]+\s*\**\s*", "", decl, count=1)
            for part in decl.split(","):
                fields.append(re.sub(r"[\s\*]|\[.*?\]", "", part))
        out[name] = fields
    return out


def test_binding_structs_match_header_layout():
    import paper_1809_07088_amd as dsx
    hs = _header_structs()
    pairs = {"dsx_model_desc": dsx.ModelDesc, "dsx_plan_info": dsx.PlanInfo,
             "dsx_kernel_stat": dsx.KernelStat, "dsx_server_config": dsx.ServerConfig,
             "dsx_request": dsx.Request, "dsx_server_stats": dsx.ServerStats}
    assert set(pairs) <= set(hs)
    for cname, py in pairs.items():
        assert [f for f, _ in py._fields_] == hs[cname], cname


# ------------------------------------------------------------------ split sites (host only)

def test_split_sites_partition_and_positions():
    from tests.helpers import discrete_displacement_model, split_model
    m = discrete_displacement_model(31, K=3)
    s = split_model(m)
    assert s.n_sites <= m.n_sites * 3
    for mu in range(m.n_sites):
        kids = np.flatnonzero(np.asarray(s.pos_id) == mu)
        # the occupancies of the split sites partition the parent's
        assert np.array_equal(s.occ[:, kids].sum(axis=1), m.occ[:, mu])
        # each split site sits at r_mu + one of the parent's displacement values
        for k in kids:
            u = s.frac[k] - m.frac[mu]
            hit = np.all(np.abs(m.disp[:, mu] - u.astype(np.float32)) <= 1e-7, axis=-1)
            assert np.array_equal(hit & (m.occ[:, mu] > 0), s.occ[:, k] > 0)


def test_split_sites_exact_against_the_exponential():
    """The split-site model, evaluated compositionally, is the displacive model with
    the exact exponential (no Taylor truncation)."""
    from tests.helpers import discrete_displacement_model, split_model
    for seed, occ in [(32, True), (33, False)]:
        m = discrete_displacement_model(seed, K=2, with_occ=occ)
        if not occ:
            m.occ = None
        s = split_model(m)
        G = O.grid_points(m.g0, m.count)[::7]
        a = O.intensity(s, G)
        b = O.intensity(m, G, -1)
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


def test_split_sites_limit():
    from tests.helpers import discrete_displacement_model
    m = discrete_displacement_model(34, K=3)
    with pytest.raises(dsx.DsxError) as e:
        dsx.split_sites(m.n, m.frac, m.b, m.disp, m.occ, 0.0, max_sites=4)
    assert e.value.status == dsx.ERR_UNSUPPORTED


def test_profile_select_arguments():
    # host-only: selecting a kernel kind touches no device state
    dsx.profile_select("recombine")
    dsx.profile_select("")
    dsx.profile_select(None)
    with pytest.raises(dsx.DsxError) as e:
        dsx.profile_select("k" * 32)
    assert e.value.status == dsx.ERR_ARG
    dsx.profile_reset()
    assert dsx.profile_read() == {}


# ------------------------------------------------------------------ binding argument checks

def test_outputs_are_written_in_place_never_copied():
    """An output the library could only fill through a temporary copy is refused."""
    ok = np.zeros((3, 4), dtype=np.float32)
    p, where = dsx._ptr_out(ok, 12)
    assert p == ok.ctypes.data and where == dsx.HOST
    for bad in (np.zeros((3, 4)), np.zeros((4, 3), dtype=np.float32).T, np.zeros(24, dtype=np.float32)[::2]):
        with pytest.raises(ValueError):
            dsx._ptr_out(bad)
    ro = np.zeros(5, dtype=np.float32)
    ro.flags.writeable = False
    with pytest.raises(ValueError):
        dsx._ptr_out(ro)


def test_array_sizes_are_checked_before_the_call():
    with pytest.raises(ValueError):
        dsx._ptr_out(np.zeros(11, dtype=np.float32), 12)
    with pytest.raises(ValueError):
        dsx._ptr_where(np.zeros((2, 5)), 11)
    p, where, keep = dsx._ptr_where(np.zeros((2, 5)), 10)    # inputs may be converted
    assert keep.dtype == np.float32 and where == dsx.HOST


def test_point_filter_output_must_hold_every_point():
    # checked in the binding, before the library is called (no model is needed)
    with pytest.raises(ValueError):
        dsx.filter_points(0, 2, np.zeros((3, 3)), np.zeros(2, dtype=np.float32))
