"""The C-ABI library loads, exports every function include/dl.h declares, and
rejects invalid arguments on the host before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1509_05054_amd import dl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(dl_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_function():
    lib = dl.lib()
    declared = _header_functions()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(dl.SIGNATURES), declared ^ set(dl.SIGNATURES)


def test_abi_version_and_status_strings():
    assert dl.lib().dl_abi_version() == 1
    assert dl.status_string(0) == "DL_OK"
    assert "workspace" in dl.status_string(-2)


@pytest.mark.parametrize("bad", [
    dict(p=6),            # not a multiple of 4
    dict(p=260),          # above 256
    dict(n=0), dict(n=1025), dict(m=0), dict(s=0), dict(s=17),
    dict(s=40, n=32),     # s > n
    dict(group_size=0), dict(precision=7), dict(rule=3),
])
def test_invalid_parameters_are_rejected(bad):
    kw = dict(p=64, n=256, m=1000, s=6)
    kw.update(bad)
    prm = dl.Params(**kw)
    assert dl.lib().dl_workspace_size(prm.ref()) == 0
    rc = dl.lib().dl_omp(prm.ref(), None, None, None, None, None, 0, None)
    assert rc == dl.DL_EINVAL


def test_params_default_and_workspace_size():
    c = dl._Params()
    assert dl.lib().dl_params_default(ctypes.byref(c), 64, 256, 16384, 6) == dl.DL_OK
    assert (c.group_size, c.precision, c.rule) == (256, 0, 0)
    assert abs(c.pivot_fp64_threshold - 1e-6) < 1e-12
    prm = dl.Params(64, 256, 16384, 6)
    size = dl.workspace_size(prm)
    # at least G, D^T Y, E and the CSR arrays
    assert size >= 4 * (256 * 256 + 16384 * 256 + 16384 * 64) + 4 * 2 * 16384 * 6


def test_null_and_misaligned_pointers_rejected_before_launch():
    prm = dl.Params(16, 32, 64, 3)
    L = dl.lib()
    fake = ctypes.c_void_p(0x1000)
    odd = ctypes.c_void_p(0x1002)
    # null dictionary
    assert L.dl_omp(prm.ref(), None, fake, fake, fake, fake, 1 << 30, None) == dl.DL_EINVAL
    # misaligned workspace (needs 256 bytes)
    assert L.dl_omp(prm.ref(), fake, fake, fake, fake, ctypes.c_void_p(0x1010), 1 << 30,
                    None) == dl.DL_EINVAL
    # misaligned float4 operand
    assert L.dl_iterate(prm.ref(), odd, fake, 1, fake, fake, fake, fake, 1 << 30,
                        None) == dl.DL_EINVAL
    # workspace too small
    assert L.dl_omp(prm.ref(), fake, fake, fake, fake, fake, 16, None) == dl.DL_EWORKSPACE
    # negative iteration count
    assert L.dl_iterate(prm.ref(), fake, fake, -1, fake, fake, fake, fake, 1 << 30,
                        None) == dl.DL_EINVAL


def _fake_problem(**kw):
    pb = dl._Problem()
    q = dict(p=16, n=32, m=100, s=3)
    q.update({k: v for k, v in kw.items() if k in ("p", "n", "m", "s")})
    pb.prm = dl.Params(**q).c()
    if "group_size" in kw:
        pb.prm.group_size = kw["group_size"]
    if "precision" in kw:
        pb.prm.precision = kw["precision"]
    for name in ("Y", "D", "X_idx", "X_val", "rmse"):
        setattr(pb, name, 0x100000)
    return pb


def test_batched_calls_validate_on_the_host():
    L = dl.lib()
    good = (dl._Problem * 2)(_fake_problem(), _fake_problem(p=64, n=256, m=5000, s=6))
    size = L.dl_batch_workspace_size(good, 2)
    singles = sum(dl.workspace_size(dl.Params(p, n, m, s))
                  for p, n, m, s in ((16, 32, 100, 3), (64, 256, 5000, 6)))
    assert size >= singles
    assert L.dl_batch_workspace_size(good, 0) == 0
    for bad in (dict(group_size=8), dict(precision=dl.PREC_BF16), dict(p=6), dict(s=0)):
        arr = (dl._Problem * 2)(_fake_problem(), _fake_problem(**bad))
        assert L.dl_batch_workspace_size(arr, 2) == 0, bad
        assert L.dl_iterate_batched(arr, 2, 1, ctypes.c_void_p(0x1000), 1 << 40, None) \
            == dl.DL_EINVAL, bad
    ws = ctypes.c_void_p(0x1000)
    assert L.dl_iterate_batched(good, 2, 1, ws, 256, None) == dl.DL_EWORKSPACE
    assert L.dl_iterate_batched(good, 2, -1, ws, 1 << 40, None) == dl.DL_EINVAL
    assert L.dl_iterate_batched(good, 2, 1, ctypes.c_void_p(0x1010), 1 << 40, None) == dl.DL_EINVAL
    assert L.dl_autotune(good, 2, 0, ws, 1 << 40, None) == dl.DL_EINVAL
    assert L.dl_autotune(good, 2, 3, ws, 256, None) == dl.DL_EWORKSPACE
    misaligned = (dl._Problem * 1)(_fake_problem())
    misaligned[0].D = 0x100004
    assert L.dl_iterate_batched(misaligned, 1, 1, ws, 1 << 40, None) == dl.DL_EINVAL


def test_rmse_noalloc_rejects_bad_arguments_on_the_host():
    """Validation happens before the scratch is looked up or anything runs."""
    ok = dl.Params(64, 256, 100, 6)
    assert dl.lib().dl_rmse_noalloc(ok.ref(), None, None, None, None, None, None) == dl.DL_EINVAL
    bad = dl.Params(64, 256, 0, 6)
    assert dl.lib().dl_rmse_noalloc(bad.ref(), None, None, None, None, None, None) == dl.DL_EINVAL
