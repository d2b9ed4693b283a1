"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/pmg.h, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re

import pytest

import paper_1808_03595_amd as pmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pmg.LIB_PATH):
        from paper_1808_03595_amd import build
        build.build()
    return pmg.lib()


def declared_names():
    src = open(os.path.join(ROOT, "include", "pmg.h")).read()
    return sorted(set(re.findall(r"\b(pmg_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_names()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
        assert n in pmg.SIGNATURES, n


def test_invalid_mesh_arguments(lib):
    h = ctypes.c_void_p()
    bad = [
        (0, 1, 1, 4, 1.0, 1.0),      # no elements
        (2, 2, 2, 0, 1.0, 1.0),      # p < 1
        (2, 2, 2, 49, 1.0, 1.0),     # p above the maximum degree
        (2, 2, 2, 4, -1.0, 1.0),     # lambda < 0
        (2, 2, 2, 4, float("nan"), 1.0),
        (2, 2, 2, 4, 1.0, 0.5),      # stretch < 1
    ]
    for args in bad:
        rc = lib.pmg_create_mesh(*args, ctypes.byref(h))
        assert rc == -1, args
        assert lib.pmg_last_error()
    assert lib.pmg_create_mesh(2, 2, 2, 4, 1.0, 1.0, None) == -1
    w = (ctypes.c_double * 2)(0.5, 0.0)
    ok = (ctypes.c_double * 2)(0.5, 0.5)
    assert lib.pmg_create_mesh_widths(2, 2, 2, 4, 1.0, w, ok, ok, ctypes.byref(h)) == -1
    assert lib.pmg_create_mesh_widths(2, 2, 2, 4, 1.0, None, ok, ok, ctypes.byref(h)) == -1


def test_invalid_boundary_kinds(lib):
    """Boundary kinds are checked before any device work (Sec. 3.3 kinds:
    0 Dirichlet, 1 Neumann, 2 periodic on both sides of a direction)."""
    h = ctypes.c_void_p()
    w3 = (ctypes.c_double * 3)(0.3, 0.3, 0.4)
    w2 = (ctypes.c_double * 2)(0.5, 0.5)
    bad = [
        (w3, (0, 0, 3, 0, 0, 0), 1.0),    # unknown kind
        (w3, (2, 0, 0, 0, 0, 0), 1.0),    # periodic on one side only
        (w3, (1, 1, 1, 1, 1, 1), 0.0),    # no Dirichlet side and lambda = 0: singular
        (w3, (2, 2, 1, 1, 2, 2), 0.0),
        (w2, (2, 2, 0, 0, 0, 0), 1.0),    # periodic direction with 2 elements
    ]
    for w, kinds, lam in bad:
        k = (ctypes.c_int * 6)(*kinds)
        n = len(w)
        assert lib.pmg_create_mesh_bc(n, 3, 3, 4, lam, w, w3, w3, k, ctypes.byref(h)) == -1, kinds
        assert lib.pmg_last_error()
    assert lib.pmg_create_mesh_bc(3, 3, 3, 4, 1.0, w3, w3, w3, None, ctypes.byref(h)) == -1


def test_null_handles_and_pointers(lib):
    L = ctypes.c_int()
    n = ctypes.c_int64()
    assert lib.pmg_num_levels(None, ctypes.byref(L)) == -1
    assert lib.pmg_skeleton_len(None, 0, ctypes.byref(n)) == -1
    assert lib.pmg_apply_condensed_op(None, 0, 0, None, None, None) == -1
    assert lib.pmg_schwarz_smooth(None, 0, 0, None, None, 1.0, None) == -1
    assert lib.pmg_vcycle(None, 0, None, None, None) == -1
    assert lib.pmg_pcg_solve(None, None, None, 1e-10, 10, 0, None, None) == -1
    assert lib.pmg_pcg_solve_dirichlet(None, None, None, None, 1e-10, 10, 0, None, None) == -1
    assert lib.pmg_lift_dirichlet(None, None, None, None, None) == -1
    assert lib.pmg_set_boundary(None, None, None, None) == -1
    assert lib.pmg_set_cycle(None, 0, 1e-8, 10) == -1
    lib.pmg_destroy_mesh(None)                    # no-op


def test_mlp_arguments(lib):
    assert lib.pmg_mlp_nparams(4) == 64 * 3 + 64 + 64 * 64 + 64 + 4 * 64 + 4
    assert lib.pmg_mlp_forward(None, None, None, None, 1, 4, None) == -1
    assert lib.pmg_mlp_adam(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None) == -1
    assert lib.pmg_mlp_adam(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1
    # the allocation-free backward pass: null pointers, then a batch whose
    # deltas exceed its fixed scratch (rejected before any device call)
    assert lib.pmg_mlp_backward_noalloc(None, None, None, None, None, 1, 4, None) == -1
    fake = ctypes.c_void_p(0x1000)
    big = (1 << 21) // (128 + 4) + 1
    assert lib.pmg_mlp_backward_noalloc(fake, fake, fake, fake, fake, big, 4, None) == -4
    assert b"scratch" in lib.pmg_last_error()


def test_binding_names_match_c_abi():
    # every Python function of the binding is the C entry point without "pmg_"
    for n in declared_names():
        short = n[len("pmg_"):]
        if short in ("last_error", "destroy_mesh"):
            continue
        assert hasattr(pmg, short) or hasattr(pmg.Mesh, short), short
