"""Host-side checks of the HIP library: it builds for gfx950, loads, exports every
entry point that include/rsfgp.h declares, and rejects bad arguments before
touching the device (no compute calls: these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1603_08057_amd import _lib, build
    if not os.path.exists(_lib.library_path()):
        build.build()
    return _lib.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rsfgp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rsf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["rsf_factor_create", "rsf_factor_destroy", "rsf_logdet", "rsf_solve", "rsf_apply",
                     "rsf_apply_sqrt", "rsf_loglik", "rsf_grad", "rsf_last_error", "rsf_opts_default",
                     "rsf_tree_export", "rsf_skeleton_export"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_opts_defaults(lib):
    from paper_1603_08057_amd._lib import Options
    o = Options()
    assert lib.rsf_opts_default(C.byref(o)) == 0
    assert (o.n_prox, o.prox_rings, o.r_near, o.prox_r_in, o.prox_r_out, o.rq_alpha, o.mem_cap_bytes) == (
        256, 4, 1.8, 1.75, 2.45, 1.0, 0)
    assert lib.rsf_opts_default(None) == -1


def _create(lib, pts, n, theta, p=3, kernel=1, eps=1e-6, leaf=64):
    h = C.c_void_p()
    th = (C.c_double * len(theta))(*theta)
    rc = lib.rsf_factor_create(pts, n, th, p, kernel, eps, leaf, None, None, C.byref(h))
    return rc, h


def test_invalid_arguments_are_rejected_before_any_device_call(lib):
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert _create(lib, None, 10, [0.1, 1.0, 1e-4])[0] == -1
    assert _create(lib, fake, 0, [0.1, 1.0, 1e-4])[0] == -1
    assert _create(lib, fake, 10, [0.1, 1.0, 1e-4], p=2)[0] == -1
    assert _create(lib, fake, 10, [0.1, 1.0, 1e-4], kernel=7)[0] == -1
    assert _create(lib, fake, 10, [0.1, 1.0, 1e-4], eps=0.0)[0] == -1
    assert _create(lib, fake, 10, [0.1, 1.0, 1e-4], leaf=0)[0] == -1
    assert _create(lib, fake, 10, [-0.1, 1.0, 1e-4])[0] == -1
    assert _create(lib, fake, 10, [float("nan"), 1.0, 1e-4])[0] == -6
    assert _create(lib, fake, 10, [0.1, 1.0, 1e-4], eps=float("inf"))[0] == -6
    assert b"eps" in lib.rsf_last_error()


def test_null_handles(lib):
    lib.rsf_factor_destroy(None)
    out = C.c_double()
    assert lib.rsf_logdet(None, C.byref(out)) == -1
    assert lib.rsf_solve(None, None, None, 1, 1, None) == -1
    assert lib.rsf_loglik(None, None, C.byref(out), None, None) == -1
    g = (C.c_double * 3)()
    assert lib.rsf_grad(None, None, 1e-6, 0, g, None, None) == -1
    assert len(lib.rsf_last_error()) > 0


def test_binding_fails_loudly_without_a_device(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    import paper_1603_08057_amd as R
    with pytest.raises(RuntimeError):
        R.Factor([[0.0, 0.0], [1.0, 1.0]], (0.1, 1.0, 1e-4))


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus 2 exits with status 2 and says why,
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
