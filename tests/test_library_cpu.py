"""Host-side checks of the HIP library that need no GPU: the shared library
loads, exports every entry point declared in include/pthr.h, and validates
parameters (no compute calls)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_2605_25872_amd import pthr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pthr.h")).read()
    return sorted(set(re.findall(r"\b(pthr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pthr.LIB_PATH):
        from paper_2605_25872_amd import build
        build.build()
    return pthr.library()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 25
    assert sorted(pthr.EXPORTED) == declared
    for name in declared:
        assert getattr(lib, name) is not None


def _create(lib, **kw):
    args = dict(L=8, n_samples=4, n_replicas=4, n_temps=20, n_reservoir=4)
    args.update(kw)
    p = pthr.make_params(**args)
    ctx = ctypes.c_void_p()
    rc = lib.pthr_create(ctypes.byref(p), ctypes.byref(ctx))
    msg = lib.pthr_create_error().decode()
    if rc == 0:
        lib.pthr_destroy(ctx)
    return rc, msg, p


def test_validation(lib):
    assert _create(lib)[0] == pthr.PTHR_OK
    rc, msg, _ = _create(lib, L=3)
    assert rc == pthr.PTHR_EUNSUPPORTED and "odd L" in msg
    assert _create(lib, n_replicas=3)[0] == pthr.PTHR_EINVAL
    assert _create(lib, n_temps=1)[0] == pthr.PTHR_EINVAL
    assert _create(lib, n_samples=0)[0] == pthr.PTHR_EINVAL
    assert _create(lib, L=40)[0] == pthr.PTHR_EINVAL
    assert _create(lib, sweeps_per_emcs=257)[0] == pthr.PTHR_EINVAL
    assert _create(lib, local_update="micsa")[0] == pthr.PTHR_OK
    assert _create(lib, local_update="micsa", micsa_refresh=3)[0] == pthr.PTHR_OK
    assert _create(lib, local_update="micsa", micsa_refresh=257)[0] == pthr.PTHR_EINVAL
    rc, msg, _ = _create(lib, L=16, n_temps=64, precision="fp32")
    assert rc == pthr.PTHR_EUNSUPPORTED and "LDS" in msg
    bad = pthr.make_params(8, 4, 4, 20, 4)
    bad.local_update = 3
    ctx = ctypes.c_void_p()
    assert lib.pthr_create(ctypes.byref(bad), ctypes.byref(ctx)) == pthr.PTHR_EINVAL
    assert lib.pthr_state_bytes(ctypes.byref(bad)) == 0


def test_sizes_of_the_headline_workload(lib):
    p = pthr.make_params(16, 1024, 4, 36, 4, precision="fp32")
    # 6 spin words of 32 clones per site, float couplings: ~154 MB for 1024 samples
    assert 150e6 < lib.pthr_state_bytes(ctypes.byref(p)) < 160e6
    assert lib.pthr_lds_bytes(ctypes.byref(p)) <= 160 * 1024
    V = 16 ** 3
    assert lib.pthr_obs_bytes(ctypes.byref(p)) >= 256 + 8 * 1024 * 36 * 6 + 8 * 36 * (V + 1)


def test_calls_before_init_fail_cleanly(lib):
    p = pthr.make_params(4, 1, 2, 8, 0)
    ctx = ctypes.c_void_p()
    assert lib.pthr_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    try:
        assert lib.pthr_sweep(ctx, 1, 0, None) == pthr.PTHR_ESTATE
        assert b"not initialised" in lib.pthr_last_error(ctx)
        assert lib.pthr_run(ctx, 1, None, None) == pthr.PTHR_ESTATE
    finally:
        lib.pthr_destroy(ctx)


def test_group_argument_checks(lib):
    """Group creation rejects bad arguments before touching the GPU."""
    grp = ctypes.c_void_p()
    assert lib.pthr_group_create(None, 1, ctypes.byref(grp)) == pthr.PTHR_EINVAL
    p = pthr.make_params(4, 1, 2, 8, 0)
    ctx = ctypes.c_void_p()
    assert lib.pthr_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    try:
        one = (ctypes.c_void_p * 1)(ctx.value)
        assert lib.pthr_group_create(one, 0, ctypes.byref(grp)) == pthr.PTHR_EINVAL
        assert lib.pthr_group_create(one, 65, ctypes.byref(grp)) == pthr.PTHR_EINVAL
        twice = (ctypes.c_void_p * 2)(ctx.value, ctx.value)
        assert lib.pthr_group_create(twice, 2, ctypes.byref(grp)) == pthr.PTHR_EINVAL
        assert b"twice" in lib.pthr_create_error()
        holes = (ctypes.c_void_p * 2)(ctx.value, None)
        assert lib.pthr_group_create(holes, 2, ctypes.byref(grp)) == pthr.PTHR_EINVAL
        assert grp.value is None
        assert lib.pthr_group_run(None, 1, None, 0, None) == pthr.PTHR_EINVAL
    finally:
        lib.pthr_destroy(ctx)


def test_default_sites_per_work_item(lib):
    """FP32 batches of two or more samples per CU (512 on an MI355X, also the
    size assumed where no device is visible) whose reservoir ends in a
    16-clone word default to 4 sites per work-item (two sites of a colour
    share one pass over that word) where that leaves 256 or more work-items;
    other contexts take the smallest chunk with a compiled kernel."""
    def threads(L, S, NERG, precision):
        p = pthr.make_params(L, S, 4, 10, NERG, precision=precision)
        ctx = ctypes.c_void_p()
        assert lib.pthr_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
        try:
            sch = pthr.Schedule()
            assert lib.pthr_get_schedule(ctx, ctypes.byref(sch)) == 0
            return sch.threads_per_sample
        finally:
            lib.pthr_destroy(ctx)
    assert threads(12, 512, 4, "fp32") == 448   # 1728 sites, 16 reservoir clones: 4 per work-item
    assert threads(12, 128, 4, "fp32") == 896   # small batch: more waves per sample
    assert threads(12, 512, 3, "fp32") == 896   # 12 reservoir clones: 2 per work-item
    assert threads(12, 512, 4, "fp64") == 896
    assert threads(10, 512, 4, "fp32") == 256   # 250 work-items of 4 sites: 4 waves
    assert threads(8, 512, 4, "fp32") == 256    # 128 work-items of 4 would be 2 waves
    assert threads(16, 512, 4, "fp32") == 1024


def test_schedule_defaults_and_checks(lib):
    """The default schedule decides FP64 tests against the float bound first
    (exp_filter = 1); set_schedule accepts 0 and refuses other values, and a
    refused schedule leaves the previous one in place."""
    p = pthr.make_params(8, 4, 4, 20, 4)
    ctx = ctypes.c_void_p()
    assert lib.pthr_create(ctypes.byref(p), ctypes.byref(ctx)) == 0
    try:
        sch = pthr.Schedule()
        assert lib.pthr_get_schedule(ctx, ctypes.byref(sch)) == 0
        assert sch.exp_filter == 1 and sch.exp_early_out == 0 and sch.clone_split in (1, 2, 4)
        sch.exp_filter = 0
        assert lib.pthr_set_schedule(ctx, ctypes.byref(sch)) == 0
        sch.exp_filter = 2
        assert lib.pthr_set_schedule(ctx, ctypes.byref(sch)) == pthr.PTHR_EINVAL
        assert b"exp_filter" in lib.pthr_last_error(ctx)
        back = pthr.Schedule()
        assert lib.pthr_get_schedule(ctx, ctypes.byref(back)) == 0
        assert back.exp_filter == 0
        # the reservoir sweeps beside the Houdayer step: off by default, 0 or 1
        assert back.overlap_reservoir == 0
        back.overlap_reservoir = 1
        assert lib.pthr_set_schedule(ctx, ctypes.byref(back)) == 0
        back.overlap_reservoir = 2
        assert lib.pthr_set_schedule(ctx, ctypes.byref(back)) == pthr.PTHR_EINVAL
        assert b"overlap_reservoir" in lib.pthr_last_error(ctx)
    finally:
        lib.pthr_destroy(ctx)
