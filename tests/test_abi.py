"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2403_16095_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "cgsr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgsr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libcgsr.so is not built; run __graft_entry__.build()")
    return B.lib()


def test_every_declared_symbol_is_exported(lib):
    decl = declared_symbols()
    assert len(decl) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {l.split()[-1] for l in out.stdout.splitlines() if " T " in l}
    missing = [s for s in decl if s not in exported]
    assert not missing, missing
    assert set(decl) == set(B.EXPORTED)
    for s in decl:
        assert hasattr(lib, s)


def test_version_and_defaults(lib):
    assert "gfx950" in B.cgsr_version()
    s = B.cgsr_default_settings()
    assert s.sync_capacity == 1 and s.timing == 0


def test_host_side_argument_checks(lib):
    # every one of these fails before any device work is enqueued
    assert lib.cgsr_render(None, None, 1, None, None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    assert "NULL" in B.cgsr_last_error()
    assert lib.cgsr_backward(None, None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_tracking_loss_grad(0, 10, None, None, None, None, 1.0, 1.0, None, None, None,
                                       None) == B.CGSR_ERR_INVALID_ARG
    good = B.cgsr_adam_params(0.1, 0.1, 0.9, 0.999, 1e-8)
    bad_beta = B.cgsr_adam_params(0.1, 0.1, 1.5, 0.999, 1e-8)
    assert lib.cgsr_pose_adam_step(0, None, None, None, C.byref(good), None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_pose_adam_step(1, 8, 8, 8, C.byref(bad_beta), None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_pose_adam_step(1, 8, 8, 8, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_tracking_step(None, None, 1, None, None, None, None, 1.0, 1.0, None, None, None, None,
                                  None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_debug_tile_order(None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    # the autotuners check their arguments before timing anything
    assert lib.cgsr_autotune_render(None, None, 1, None, None, None, None, None, None, None, 3, None,
                                    None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_autotune_tracking(None, None, 1, None, None, None, None, 3, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_render_nu(None, None, 1, None, None, None, None, None, None, None,
                              None) == B.CGSR_ERR_INVALID_ARG
    # sensor depth is required; nu_sum and nu_count come together
    assert lib.cgsr_render_nu(8, None, 1, None, None, None, None, None, 8, 8, None) == B.CGSR_ERR_INVALID_ARG
    dep = (C.c_void_p * 1)(8)
    assert lib.cgsr_render_nu(8, None, 1, None, None, dep, None, None, 8, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_nu_prune(-1, None, None, 0.025, 0.01, None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_nu_prune(4, None, None, 0.025, 0.01, None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_nu_prune(4, 8, 8, -1.0, 0.01, None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_nu_prune(4, 8, 8, 0.025, 1.0, None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_nu_prune(4, 8, 8, 0.025, 0.0, None, None, None, None) == B.CGSR_ERR_INVALID_ARG
    hp = B.cgsr_gaussian_adam_params(1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 0.9, 0.999, 1e-15)
    gg = B.cgsr_gaussian_grads(8, 8, 8, 8, 8)
    assert lib.cgsr_gaussian_adam_step(-1, C.byref(gg), C.byref(gg), 8, 8, C.byref(hp), None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_gaussian_adam_step(4, None, C.byref(gg), 8, 8, C.byref(hp), None) == B.CGSR_ERR_INVALID_ARG
    bad_hp = B.cgsr_gaussian_adam_params(1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1.0, 0.999, 1e-15)
    assert lib.cgsr_gaussian_adam_step(4, C.byref(gg), C.byref(gg), 8, 8, C.byref(bad_hp), None) == B.CGSR_ERR_INVALID_ARG
    neg_lr = B.cgsr_gaussian_adam_params(-1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 0.9, 0.999, 1e-15)
    assert lib.cgsr_gaussian_adam_step(4, C.byref(gg), C.byref(gg), 8, 8, C.byref(neg_lr), None) == B.CGSR_ERR_INVALID_ARG
    part = B.cgsr_gaussian_grads(8, None, 8, 8, 8)
    assert lib.cgsr_gaussian_adam_step(4, C.byref(part), C.byref(gg), 8, 8, C.byref(hp), None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_state_check(None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_get_stats(None, None, None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_state_reserve(None, 1, 1, 1, 1) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_state_destroy(None) == B.CGSR_OK
    bad = B.cgsr_settings(2, 0, 1, 1)
    out = C.c_void_p()
    assert lib.cgsr_state_create(C.byref(bad), C.byref(out)) == B.CGSR_ERR_INVALID_ARG
    assert out.value is None
    bad_ppl = B.cgsr_settings(1, 0, 3, 1)
    assert lib.cgsr_state_create(C.byref(bad_ppl), C.byref(out)) == B.CGSR_ERR_INVALID_ARG
    bad_count = B.cgsr_settings(1, 0, 1, 1, 2)
    assert lib.cgsr_state_create(C.byref(bad_count), C.byref(out)) == B.CGSR_ERR_INVALID_ARG
    assert B.cgsr_default_settings().count_work == 1


def test_binding_raises_with_message(lib):
    with pytest.raises(B.CgsrError) as e:
        B.cgsr_tracking_loss_grad(0, 0, 0, 0, 0, 0, 1.0, 1.0, 0, 0, None, None)
    assert e.value.status == B.CGSR_ERR_INVALID_ARG


def test_management_and_sh_argument_checks(lib):
    ga = B.cgsr_gaussian_arrays(8, 16, 24, 32, 40, None, 0)
    cam = B.cgsr_camera(64, 48, 60.0, 60.0, 32.0, 24.0)
    n_out = C.c_int64(-7)
    spawn = lambda arr, n, cap, stride=1, c=C.byref(cam): lib.cgsr_spawn_gaussians(
        arr, n, cap, c, 8, 8, 8, None, 0.5, stride, 0.0, C.byref(n_out), None)
    assert spawn(None, 0, 10) == B.CGSR_ERR_INVALID_ARG
    assert spawn(C.byref(ga), 11, 10) == B.CGSR_ERR_INVALID_ARG          # n > capacity
    assert spawn(C.byref(ga), 0, 10, stride=0) == B.CGSR_ERR_INVALID_ARG
    assert spawn(C.byref(ga), 0, 10, c=None) == B.CGSR_ERR_INVALID_ARG
    no_colour = B.cgsr_gaussian_arrays(8, 16, 24, 32, None, None, 0)
    assert spawn(C.byref(no_colour), 0, 10) == B.CGSR_ERR_INVALID_ARG
    bad_deg = B.cgsr_gaussian_arrays(8, 16, 24, 32, None, 48, 4)
    assert spawn(C.byref(bad_deg), 0, 10) == B.CGSR_ERR_INVALID_ARG
    assert n_out.value == -7, "a rejected call writes nothing"
    other = B.cgsr_gaussian_arrays(108, 116, 124, 132, 140, None, 0)
    sh_set = B.cgsr_gaussian_arrays(208, 216, 224, 232, None, 248, 1)
    shared = B.cgsr_gaussian_arrays(108, 16, 124, 132, 140, None, 0)     # log_scales shared with ga
    z = (C.c_void_p * 1)()
    w = (C.c_int32 * 1)()
    compact = lambda src, dst, n=4, keep=8, k=0: lib.cgsr_compact_gaussians(
        n, keep, C.byref(src), C.byref(dst), k, z, z, w, C.byref(n_out), None)
    assert compact(ga, shared) == B.CGSR_ERR_INVALID_ARG
    assert compact(ga, sh_set) == B.CGSR_ERR_INVALID_ARG                 # colour layouts differ
    assert compact(ga, other, keep=None) == B.CGSR_ERR_INVALID_ARG
    assert compact(ga, other, k=13) == B.CGSR_ERR_INVALID_ARG
    assert compact(ga, other, n=-1) == B.CGSR_ERR_INVALID_ARG
    # the allocation-free variant: same checks, and n beyond its fixed scratch
    compact0 = lambda src, dst, n=4, keep=8, k=0: lib.cgsr_compact_gaussians_noalloc(
        n, keep, C.byref(src), C.byref(dst), k, z, z, w, C.byref(n_out), None)
    assert compact0(ga, shared) == B.CGSR_ERR_INVALID_ARG
    assert compact0(ga, other, keep=None) == B.CGSR_ERR_INVALID_ARG
    assert compact0(ga, other, n=-1) == B.CGSR_ERR_INVALID_ARG
    assert compact0(ga, other, n=(1 << 26) + 1) == B.CGSR_ERR_INVALID_ARG
    assert "exceeds its fixed scratch" in B.cgsr_last_error()
    dens = lambda src, dst, n=4, normals=8: lib.cgsr_densify_gaussians(
        n, 8, 8, 1e-4, 0.01, normals, C.byref(src), C.byref(dst), 10, C.byref(n_out), None)
    assert dens(ga, other, normals=None) == B.CGSR_ERR_INVALID_ARG
    assert dens(ga, ga) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_set_densify_stats(None, 8, 8) == B.CGSR_ERR_INVALID_ARG
    # view-dependent colour: Adam needs both sh arrays and a valid degree
    hp = B.cgsr_gaussian_adam_params(1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 0.9, 0.999, 1e-15, 1e-4, 4)
    with_sh = B.cgsr_gaussian_grads(8, 8, 8, 8, None, 8)
    without = B.cgsr_gaussian_grads(8, 8, 8, 8, 8, None)
    assert lib.cgsr_gaussian_adam_step(4, C.byref(with_sh), C.byref(without), 8, 8, C.byref(hp),
                                       None) == B.CGSR_ERR_INVALID_ARG
    assert lib.cgsr_gaussian_adam_step(4, C.byref(with_sh), C.byref(with_sh), 8, 8, C.byref(hp),
                                       None) == B.CGSR_ERR_INVALID_ARG   # degree 4
