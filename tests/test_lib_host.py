"""Host-side logic of libfewha on the CPU: exported symbols, set-up tables
against the oracle (db3 filter, prior D, sensor masks, exact Jacobi diagonal
J of eq. precond), argument validation.  No compute call runs here."""

import os
import re
from ctypes import c_void_p

import numpy as np
import pytest

from synthetic import get_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "fewha.h")).read()
    names = set(re.findall(r"FEWHA_API\s+[\w\s\*]+?\b(fewha_\w+)\s*\(", hdr))
    assert len(names) >= 20
    import ctypes
    so = ctypes.CDLL(lib._abi.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(so, n)]
    assert not missing, missing
    assert names == set(lib._abi.EXPORTED)


def test_filter_matches_oracle(lib):
    from oracle.wavelet import daubechies_filter
    ctx = lib.Context(get_config("tiny"), device=-1)
    h = ctx.get_table(lib._abi.FEWHA_TABLE_FILTER)
    assert np.allclose(h, daubechies_filter(3), atol=1e-15, rtol=0)


@pytest.mark.parametrize("name", ["tiny", "small", "mid"])
def test_prior_mask_and_preconditioner_match_oracle(lib, systems, name):
    S = systems(name)
    ctx = lib.Context(get_config(name), device=-1)
    assert np.array_equal(ctx.get_table(lib._abi.FEWHA_TABLE_PRIOR), S.D)
    mask = np.concatenate([m.ravel() for m in S.geom.masks]).astype(float)
    assert np.array_equal(ctx.get_table(lib._abi.FEWHA_TABLE_MASK), mask)
    J = ctx.get_table(lib._abi.FEWHA_TABLE_PRECOND)
    assert np.allclose(J, S.preconditioner(), rtol=1e-10, atol=0)
    assert ctx.n_coeff == S.geom.n_coeff and ctx.n_slopes == sum(S.geom.n_slopes)


def test_preconditioner_with_elongation_and_tau(lib):
    from oracle.operators import System
    cfg = get_config("small")
    cfg["noise"]["alpha_eta"] = 0.6
    cfg["prior"]["tau"] = 3.0
    S = System(cfg)
    ctx = lib.Context(cfg, device=-1)
    assert np.allclose(ctx.get_table(lib._abi.FEWHA_TABLE_PRECOND), S.preconditioner(), rtol=1e-10, atol=0)


@pytest.mark.slow
def test_preconditioner_maory_like(lib, systems):
    S = systems("maory_like")
    ctx = lib.Context(get_config("maory_like"), device=-1)
    assert np.allclose(ctx.get_table(lib._abi.FEWHA_TABLE_PRECOND), S.preconditioner(), rtol=1e-10, atol=0)


def test_user_mask_is_used(lib):
    cfg = get_config("small")
    m = np.zeros((20, 20), dtype=np.uint8)
    m[2:18, 3:17] = 1
    cfg["wfs"][0]["mask"] = m
    ctx = lib.Context(cfg, device=-1)
    got = ctx.get_table(lib._abi.FEWHA_TABLE_MASK)[:400].reshape(20, 20)
    assert np.array_equal(got, m.astype(float))


def _expect(lib, status, fn):
    with pytest.raises(lib.FewhaError) as e:
        fn()
    assert e.value.status == status


def test_geometry_errors(lib):
    cfg = get_config("small")
    cfg["layers"][2]["n"] = 48  # not a power of two
    _expect(lib, -5, lambda: lib.Context(cfg, device=-1))
    cfg = get_config("small")
    cfg["wfs"][3]["theta"] = (300e-6, 0.0)  # footprint leaves the layer
    _expect(lib, -5, lambda: lib.Context(cfg, device=-1))
    cfg = get_config("small")
    cfg["layers"][0]["levels"] = 9  # deeper than log2(32)
    _expect(lib, -5, lambda: lib.Context(cfg, device=-1))
    cfg = get_config("small")
    cfg["layers"][1]["h"] = 95000.0  # above the sodium layer
    _expect(lib, -5, lambda: lib.Context(cfg, device=-1))


def test_argument_errors(lib):
    import ctypes
    a = lib._abi
    h = ctypes.c_void_p()
    assert a.fewha_create(None, -1) == -1
    assert a.fewha_create(ctypes.byref(h), -1) == 0
    assert a.fewha_set_pupil(h, -1.0, 0.1) == -1
    assert a.fewha_set_pupil(h, 8.0, 1.0) == -1
    assert a.fewha_set_wfs(h, 0, None) == -1
    assert a.fewha_set_prior(h, 0.0, 0.15, 25.0, 0.0) == -1
    assert a.fewha_set_control(h, 1.5) == -1
    assert a.fewha_finalize(h) == -4  # nothing configured
    assert b"pupil" in a.fewha_last_error(h)
    a.fewha_destroy(h)


def test_compute_on_host_only_context_is_a_state_error(lib):
    ctx = lib.Context(get_config("tiny"), device=-1)
    a = lib._abi
    x = ctypes_dummy()
    assert a.fewha_apply_M(ctx.h, x, x) == -4
    assert a.fewha_reconstruct(ctx.h, x, x, None, None, 4) == -4


def ctypes_dummy():
    import ctypes
    return ctypes.c_void_p(16)


def test_tuning_arguments_are_validated(lib):
    from ctypes import byref
    from paper_2202_11945_amd import _abi
    from paper_2202_11945_amd.fewha import _tuning
    ctx = lib.Context(get_config("tiny"), device=-1)  # finalized host-only context
    assert _abi.fewha_set_tuning(ctx.h, byref(_tuning(64))) == -4  # after finalize
    h = c_void_p()
    assert _abi.fewha_create(byref(h), -1) == 0
    for bad in (16, 96, -1, 256):
        assert _abi.fewha_set_tuning(h, byref(_tuning(bad))) == -1
    t = _tuning(32)
    t.reserved[1] = 1
    assert _abi.fewha_set_tuning(h, byref(t)) == -1
    assert _abi.fewha_set_tuning(h, byref(_tuning({"glob_fuse": 2}))) == -1
    assert _abi.fewha_set_tuning(h, byref(_tuning({"glob_fuse": 1}))) == 0
    for bad in ({"pt_split": 2}, {"pt_split": -1}, {"pt_split": 1, "pt_rows": 8}):
        assert _abi.fewha_set_tuning(h, byref(_tuning(bad))) == -1
    for ok in ({"pt_split": 1}, {"pt_split": 1, "pt_rows": 4}, {"pt_split": 0, "pt_rows": 8}):
        assert _abi.fewha_set_tuning(h, byref(_tuning(ok))) == 0
    for bad_rows in (2, 6, 16, -4):
        assert _abi.fewha_set_tuning(h, byref(_tuning({"pt_rows": bad_rows}))) == -1
    for good in (0, 32, 64, 128):
        assert _abi.fewha_set_tuning(h, byref(_tuning(good))) == 0
    for rows in (0, 4, 8):
        assert _abi.fewha_set_tuning(h, byref(_tuning({"dwt_resident": 64, "pt_rows": rows}))) == 0
    # a context runs one stream
    assert _abi.fewha_set_tuning(h, byref(_tuning({"streams": 2}))) == -1
    for one in (0, 1):
        assert _abi.fewha_set_tuning(h, byref(_tuning({"streams": one}))) == 0
    _abi.fewha_destroy(h)
    # a batch takes 1..4 streams, at most one per problem; the tuning is checked
    # before the contexts (these are host-only, so a valid tuning gets ESTATE)
    arr = (c_void_p * 2)(ctx.h.value, ctx.h.value)
    b = c_void_p()
    for bad in (-1, 3, 5):
        assert _abi.fewha_batch_create_tuned(byref(b), arr, 2, byref(_tuning({"streams": bad}))) == -1
    for ok in (0, 1, 2):
        assert _abi.fewha_batch_create_tuned(byref(b), arr, 2, byref(_tuning({"streams": ok}))) == -4


def test_photon_counts_set_the_noise(lib):
    # sigma_g^2 = 1 / n_photons (eq. NGS-noise, eq. LGS-noise): the exact
    # Jacobi diagonal, which depends on every sensor's noise weight, matches
    # the oracle's for a photon-count configuration (lowflux LGS, highflux NGS)
    from oracle.operators import System
    cfg = get_config("small")
    for w in cfg["wfs"]:
        w["photons"] = 500.0 if w["kind"] == "lgs" else 10000.0
        w["sigma"] = 123.0  # replaced by the photon counts
    S = System(cfg)
    ctx = lib.Context(cfg, device=-1)
    assert np.allclose(ctx.get_table(lib._abi.FEWHA_TABLE_PRECOND), S.preconditioner(), rtol=1e-10, atol=0)


def test_loop_and_photon_arguments(lib):
    from ctypes import byref, c_double
    a = lib._abi
    h = c_void_p()
    assert a.fewha_create(byref(h), -1) == 0
    two = (c_double * 2)(100.0, 100.0)
    assert a.fewha_set_photons(h, 2, two) == -4  # before set_wfs
    assert a.fewha_set_loop(h, 2) == -1
    assert a.fewha_set_loop(h, 1) == 0
    a.fewha_destroy(h)
    cfg = get_config("small_fit", loop="closed")
    with pytest.raises(lib.FewhaError) as e:
        lib.Context(cfg, device=-1)
    assert e.value.status == -1 and "F = I" in str(e.value)
    cfg = get_config("small")
    cfg["wfs"][0]["photons"] = 0.0
    for w in cfg["wfs"][1:]:
        w["photons"] = 100.0
    with pytest.raises(lib.FewhaError) as e:
        lib.Context(cfg, device=-1)
    assert e.value.status == -1


def test_solve_coarse_side_is_validated(lib):
    from ctypes import byref
    a = lib._abi
    h = c_void_p()
    assert a.fewha_create(byref(h), -1) == 0
    for side in (0, 1, 8, 16, 64):
        assert a.fewha_set_solve_coarse(h, side) == 0
    for side in (-1, 3, 12, 128):
        assert a.fewha_set_solve_coarse(h, side) == -1
    assert a.fewha_batch_set_solve_coarse(None, 16) == -1
    a.fewha_destroy(h)
