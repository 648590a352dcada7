"""The C ABI library without a GPU: it loads, exports every entry point that
include/hrt.h declares, and its host-only plan (hrt_plan_describe) agrees
with the oracle's independent geometry."""
import ctypes as C
import math
import os
import re

import pytest

import synth
from oracle import geometry
from paper_1604_07651_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hrt.h")).read()
    return sorted(set(re.findall(r"\b(hrt_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(n for n, _, _ in _lib.SIGNATURES) == names


def describe(desc):
    lib = _lib.load()
    info = _lib.HrtInfo()
    st = lib.hrt_plan_describe(C.byref(_lib.make_desc(desc)), C.byref(info))
    return st, info


DESCS = [synth.config_desc("c1"), synth.config_desc("c2"), synth.config_desc("c3"),
         synth.GridDesc(nt=37, nx=23, dt=0.01, x0=0.05, dx=0.03, ntau=29, nq=19,
                        tau0=0.07, dtau=0.01, q0=0.3, dq=0.021, oversample=2.5),
         synth.GridDesc(nt=16, nx=16, dt=0.01, x0=0.0, dx=0.02, ntau=16, nq=16,
                        tau0=0.0, dtau=0.01, q0=0.25, dq=(1 / 1.5 - 0.25) / 15)]


@pytest.mark.parametrize("desc", DESCS)
def test_host_plan_matches_oracle_geometry(desc):
    st, info = describe(desc)
    assert st == 0
    g = geometry.build(desc)
    for name, ref in [("T", g.T), ("X", g.X), ("alpha", g.alpha), ("beta", g.beta),
                      ("a", g.a), ("O1", g.O1), ("O2", g.O2), ("a_r", g.a_r),
                      ("dtheta0", g.dtheta0), ("drho0", g.drho0),
                      ("dtheta", g.dtheta), ("drho", g.drho), ("beta_k", g.beta_k)]:
        assert abs(getattr(info, name) - ref) <= 1e-13 * max(1.0, abs(ref)), name
    assert (info.m_theta, info.m_rho) == (g.Mtheta, g.Mrho)
    assert info.n_kept == int(g.keep.sum())
    assert info.k1_kept == math.ceil(g.Mtheta / (2 * g.sigma))
    assert info.k2_kept == math.ceil(g.Mrho / (2 * g.sigma))
    # every point's rows (in the library's placement) lie inside [row_lo, row_hi)
    crho = math.ceil(abs(math.log(g.a_r)) / g.drho) + 3
    ys = list((g.eta[g.keep] / g.drho + crho)) + list((g.rho / g.drho + crho).ravel())
    assert info.row_lo <= math.floor(min(ys)) - 1
    assert math.floor(max(ys)) + 2 < info.row_hi <= info.m_rho
    assert info.band_rows % 2 == 0 and info.n_bands * info.band_rows >= info.row_hi - info.row_lo


def test_describe_rejects_bad_grids():
    lib = _lib.load()
    base = DESCS[3]
    for bad in [base.with_(nt=3), base.with_(dq=0.0), base.with_(q0=-0.1),
                base.with_(ntau=100), base.with_(oversample=1.2), base.with_(dx=-1.0)]:
        st, _ = describe(bad)
        assert st == 1
        assert lib.hrt_last_error()
    assert lib.hrt_plan_describe(None, None) == 1


def test_status_strings_and_bad_handles():
    lib = _lib.load()
    assert lib.hrt_status_string(0) == b"ok"
    assert lib.hrt_status_string(5) == b"bad plan handle"
    # a pointer that is no live plan is refused without being dereferenced
    bogus = C.c_void_p(0x1234)
    assert lib.hrt_forward(bogus, None, None, None) == 5
    assert lib.hrt_normal(bogus, None, None, None, None) == 5
    assert lib.hrt_query(None, None) == 1
    lib.hrt_plan_destroy(bogus)   # ignored


def test_describe_accepts_tuning_flags_and_rejects_others():
    lib = _lib.load()
    info = _lib.HrtInfo()
    d = synth.config_desc("c1")
    for fl in range(128):
        assert lib.hrt_plan_describe(C.byref(_lib.make_desc(d, fl)), C.byref(info)) == 0
        # the band height the flags ask for
        want = 2 if fl & _lib.TUNE_BAND2 else 4 if fl & _lib.TUNE_BAND4 else 8
        assert info.band_rows == want
    assert lib.hrt_plan_describe(C.byref(_lib.make_desc(d, 128)), C.byref(info)) == 1
    assert lib.hrt_plan_describe(C.byref(_lib.make_desc(d, -1)), C.byref(info)) == 1


SPLITS = [(synth.config_desc("c1"), [0, 64, 256], [0, 64, 128]),
          (synth.config_desc("c1"), [0, 32, 96, 256], [0, 40, 80, 128]),
          (DESCS[3], [0, 15, 37], [0, 9, 19]),
          (synth.config_desc("c3"), [0, 768, 2048], [0, 512, 1024])]


@pytest.mark.parametrize("desc,te,qe", SPLITS)
def test_host_split_parts_match_oracle(desc, te, qe):
    """hrt_split_describe derives every part (grid, bands, geometry) as the
    oracle's independent split does."""
    from oracle import split
    from paper_1604_07651_amd import hrt
    parts = split.parts(desc, te, qe)
    for i, p in enumerate(parts):
        got = hrt.describe_part(desc, te, qe, i)
        for k in ("nt", "nx", "ntau", "nq", "q0", "dt", "dx", "x0", "tau0", "dtau", "dq"):
            assert got[k] == getattr(p.desc, k), (i, k)
        assert (got["j_lo"], got["j_hi"], got["l_lo"], got["l_hi"]) == (p.j_lo, p.j_hi, p.l_lo,
                                                                         p.l_hi)
        g = geometry.build(p.desc, (p.j_lo, p.j_hi))
        info = got["info"]
        for name, ref in [("T", g.T), ("X", g.X), ("beta", g.beta), ("a", g.a),
                          ("dtheta0", g.dtheta0), ("drho0", g.drho0)]:
            assert abs(info[name] - ref) <= 1e-13 * max(1.0, abs(ref)), (i, name)
        assert (info["m_theta"], info["m_rho"]) == (g.Mtheta, g.Mrho)
        assert info["n_kept"] == int(g.keep.sum())


def test_host_split_rejects_bad_edges():
    from paper_1604_07651_amd import hrt
    d = synth.config_desc("c1")
    for te, qe in [([0, 100, 90, 256], [0, 128]), ([0, 256], [1, 128]), ([0, 255], [0, 128]),
                   ([0, 1, 256], [0, 128])]:
        with pytest.raises(_lib.HrtError):
            for i in range((len(te) - 1) * (len(qe) - 1)):
                hrt.describe_part(d, te, qe, i)
    with pytest.raises(_lib.HrtError):
        hrt.describe_part(d, [0, 128, 256], [0, 128], 2)


def test_sector_wider_than_the_method_allows_is_refused():
    """Slownesses from 0 to 0.6 s/km over offsets to 1.5 km at 0.4 s span
    a sector whose kernel half-width reaches 1.5 rad (cos -> 0 in the
    kernel's 1/cos): the plan refuses it as a geometry error before any
    allocation."""
    lib = _lib.load()
    info = _lib.HrtInfo()
    d = synth.GridDesc(nt=5, nx=4, dt=0.1, x0=0.0, dx=0.5, ntau=4, nq=5, tau0=0.0,
                       dtau=0.1, q0=0.0, dq=0.15)
    assert lib.hrt_plan_describe(C.byref(_lib.make_desc(d)), C.byref(info)) == 2
    assert b"sector" in lib.hrt_last_error()
