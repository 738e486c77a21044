"""Host-side checks of the C ABI (no GPU): the library loads, exports every
declared symbol, its structs match the header, and every argument error that
validation catches before the first HIP call is reported."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmdmi.h")


@pytest.fixture(scope="module")
def L():
    from paper_2502_05339_amd import _lib
    return _lib.lib()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmd_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_no_extra_exports():
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2502_05339_amd", "libdmdmi.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = sorted(set(re.findall(r" T (dmd_[a-z0-9_]+)", out)))
    assert exported == _declared_functions()


def test_version_and_strings(L):
    from paper_2502_05339_amd import _lib
    assert L.dmd_abi_version() == 3
    for code in range(0, 13):
        assert len(_lib.status_string(code)) >= 2
    assert "unknown" in _lib.status_string(99)
    assert L.dmd_phi_ld(1) == 32 and L.dmd_phi_ld(150) == 160 and L.dmd_phi_ld(160) == 160


def test_struct_layout_matches_header():
    from paper_2502_05339_amd import _lib
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "dmdmi.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(dmd_fit_opts), sizeof(dmd_model), sizeof(dmd_scene));
  printf("%zu %zu %zu\n", offsetof(dmd_fit_opts, omega), offsetof(dmd_model, info), offsetof(dmd_scene, ws_bytes));
  printf("%zu %zu %zu\n", sizeof(dmd_edit), offsetof(dmd_edit, re_shift), offsetof(dmd_edit, im_scale));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = list(map(int, out))
    assert sizes[:3] == [ctypes.sizeof(_lib.FitOpts), ctypes.sizeof(_lib.ModelStruct), ctypes.sizeof(_lib.SceneStruct)]
    assert sizes[3] == _lib.FitOpts.omega.offset
    assert sizes[4] == _lib.ModelStruct.info.offset
    assert sizes[5] == _lib.SceneStruct.ws_bytes.offset
    assert sizes[6:] == [ctypes.sizeof(_lib.EditStruct), _lib.EditStruct.re_shift.offset,
                         _lib.EditStruct.im_scale.offset]


def _opts(r=10, p=4, q=1, precision="mixed", omega=0x1000):
    from paper_2502_05339_amd import fit_opts
    o = fit_opts(r, p, q, precision)
    o.omega = omega
    return o


def _ws_size(L, n, ncols, dtype, o):
    nb = ctypes.c_size_t(0)
    st = L.dmd_fit_workspace_size(n, ncols, dtype, ctypes.byref(o), ctypes.byref(nb))
    return st, nb.value


@pytest.mark.parametrize("n,ncols,r,p,expect", [
    (1000, 30, 10, 4, 0),
    (1000, 30, 31, 0, 2),      # r > m-1
    (1000, 30, 25, 10, 2),     # l > m-1
    (10, 30, 8, 4, 2),         # l > N
    (0, 30, 8, 4, 2),          # empty
    (1000, 400, 170, 10, 11),  # r beyond the eigen-solver limit
    (1000, 400, 150, 60, 11),  # l beyond the sketch limit
    (1000, 400, 150, 10, 0),   # l = 160, the largest sketch
    (1000, 400, 150, 11, 11),  # l = 161
    (1000, 400, 160, 32, 11),  # r at the eigen-solver limit, l = 192
])
def test_fit_shape_validation(L, n, ncols, r, p, expect):
    st, _ = _ws_size(L, n, ncols, 0, _opts(r, p))
    assert st == expect


def test_fit_dtype_and_enum_validation(L):
    assert _ws_size(L, 1000, 30, 1, _opts(precision="mixed"))[0] == 1       # mixed needs FP32
    assert _ws_size(L, 1000, 30, 0, _opts(precision="fp64"))[0] == 1        # fp64 needs FP64
    o = _opts()
    o.precision = 7
    assert _ws_size(L, 1000, 30, 0, o)[0] == 1
    o = _opts()
    o.dt = 0.0
    assert _ws_size(L, 1000, 30, 0, o)[0] == 1
    o = _opts(r=16, p=0, q=0, precision="fp64_exact")
    assert _ws_size(L, 8192, 64, 1, o)[0] == 0
    for trials, expect in ((-1, 1), (0, 0), (500, 0), (100000, 0), (100001, 1)):
        o = _opts()
        o.flags = 4 | 1                     # OptDMD, asynchronous: a trial budget
        o.optdmd_trials = trials
        assert _ws_size(L, 1000, 30, 0, o)[0] == expect, trials
    assert _ws_size(L, 8192, 250, 1, _opts(r=16, p=0, q=0, precision="fp64_exact"))[0] == 11


def test_autotune_fit_argument_errors(L):
    """The fit autotuner validates like dmd_fit before touching the device: no options,
    inconsistent sizes, a too small workspace."""
    m = _model_struct(n=1000, r=10)
    assert L.dmd_autotune_fit(None, 0x1000, 0x2000, 1000, 30, 1000, 1000, 0, None, 0x3000, 1 << 30,
                              ctypes.byref(m), None) == 1
    o = _opts(r=40, p=10)
    assert L.dmd_autotune_fit(None, 0x1000, 0x2000, 1000, 30, 1000, 1000, 0, ctypes.byref(o), 0x3000, 1 << 30,
                              ctypes.byref(m), None) != 0
    o = _opts(r=10, p=4)
    assert L.dmd_autotune_fit(None, 0x1000, 0x2000, 1000, 30, 1000, 1000, 0, ctypes.byref(o), 0x3000, 16,
                              ctypes.byref(m), None) == 3


def test_workspace_sizes_scale(L):
    st, small = _ws_size(L, 131072, 199, 0, _opts(150, 10, 2))
    st2, big = _ws_size(L, 6291456, 299, 0, _opts(150, 10, 2))
    assert st == st2 == 0
    # the sketch Y (N x l floats) dominates
    assert big >= 6291456 * 160 * 4
    assert small < 400 * 2 ** 20


def _model_struct(n=1000, r=10, dtype=0, ldphi=32, phi=0x10000):
    from paper_2502_05339_amd import _lib
    m = _lib.ModelStruct()
    m.n, m.r, m.dtype, m.dt, m.phi, m.ldphi = n, r, dtype, 1.0, phi, ldphi
    m.lam = m.b = m.sigma = m.kind = m.info = 0x20000
    return m


def test_fit_pointer_and_workspace_errors(L):
    o = _opts()
    m = _model_struct()
    # null X
    assert L.dmd_fit(None, None, 0x100, 1000, 30, 1000, 1000, 0, ctypes.byref(o), 0x1000, 1 << 30, ctypes.byref(m)) == 1
    # misaligned phi
    m2 = _model_struct(phi=0x10004)
    assert L.dmd_fit(None, 0x100, 0x200, 1000, 30, 1000, 1000, 0, ctypes.byref(o), 0x1000, 1 << 30,
                     ctypes.byref(m2)) == 1
    # ldphi not a multiple of 32
    m3 = _model_struct(ldphi=40)
    assert L.dmd_fit(None, 0x100, 0x200, 1000, 30, 1000, 1000, 0, ctypes.byref(o), 0x1000, 1 << 30,
                     ctypes.byref(m3)) == 1
    # model rows differ from X rows
    m4 = _model_struct(n=999)
    assert L.dmd_fit(None, 0x100, 0x200, 1000, 30, 1000, 1000, 0, ctypes.byref(o), 0x1000, 1 << 30,
                     ctypes.byref(m4)) == 2
    # leading dimension smaller than N
    assert L.dmd_fit(None, 0x100, 0x200, 1000, 30, 999, 1000, 0, ctypes.byref(o), 0x1000, 1 << 30,
                     ctypes.byref(m)) == 1
    # missing sketch
    o2 = _opts(omega=0)
    assert L.dmd_fit(None, 0x100, 0x200, 1000, 30, 1000, 1000, 0, ctypes.byref(o2), 0x1000, 1 << 30,
                     ctypes.byref(m)) == 1
    # workspace too small
    _, need = _ws_size(L, 1000, 30, 0, o)
    assert L.dmd_fit(None, 0x100, 0x200, 1000, 30, 1000, 1000, 0, ctypes.byref(o), 0x1000, need - 1,
                     ctypes.byref(m)) == 3


def test_reconstruct_validation(L):
    from paper_2502_05339_amd import _lib
    m = _model_struct(r=10)
    ks = (ctypes.c_int64 * 4)(0, 1, 2, 3)
    nb = ctypes.c_size_t(0)
    assert L.dmd_reconstruct_workspace_size(10, 4, 3, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.dmd_reconstruct_workspace_size(10, 0, 3, ctypes.byref(nb)) == 2
    assert L.dmd_reconstruct_workspace_size(10, 4, 9, ctypes.byref(nb)) == 1
    # FP64 mode on an FP32 model
    assert L.dmd_reconstruct(None, ctypes.byref(m), ks, 4, 0, 0x1000, 1000, 0x2000, 1 << 20) == 1
    # K = 0
    assert L.dmd_reconstruct(None, ctypes.byref(m), ks, 0, 1, 0x1000, 1000, 0x2000, 1 << 20) == 2
    # ldu < N
    assert L.dmd_reconstruct(None, ctypes.byref(m), ks, 4, 1, 0x1000, 999, 0x2000, 1 << 20) == 1
    # small workspace
    L.dmd_reconstruct_workspace_size(10, 4, 1, ctypes.byref(nb))
    assert L.dmd_reconstruct(None, ctypes.byref(m), ks, 4, 1, 0x1000, 1000, 0x2000, nb.value - 1) == 3
    # rank beyond the reconstruction's register tile
    big = _model_struct(r=200, ldphi=224)
    assert L.dmd_reconstruct(None, ctypes.byref(big), ks, 4, 1, 0x1000, 1000, 0x2000, 1 << 20) == 11
    # non-finite time
    ts = (ctypes.c_double * 2)(0.0, float("nan"))
    assert L.dmd_integrate(None, ctypes.byref(m), ts, 2, 1, 0x1000, 1000, 0x2000, 1 << 20) == 1
    assert _lib.DMD_OK == 0


def test_project_and_loss_validation(L):
    m = _model_struct(r=10)
    nb = ctypes.c_size_t(0)
    assert L.dmd_project_workspace_size(1000, 10, ctypes.byref(nb)) == 0
    assert L.dmd_project(None, ctypes.byref(m), None, 0x100, 0x1000, 1 << 20) == 1
    assert L.dmd_project(None, ctypes.byref(m), 0x100, 0x200, 0x1000, 0) == 3
    assert L.dmd_loss_grad_workspace_size(1000, 10, 20, 0, ctypes.byref(nb)) == 0
    ks = (ctypes.c_int64 * 2)(0, 1)
    assert L.dmd_loss_grad(None, ctypes.byref(m), 0x100, 0x100, 0x100, 999, ks, 2, 0x300, 0x1000, 1 << 20) == 1
    assert L.dmd_loss_grad(None, ctypes.byref(m), 0x100, 0x100, 0x100, 1000, ks, 2, 0x300, 0x1000, 0) == 3


def test_batched_validation(L):
    from paper_2502_05339_amd import _lib
    sc = (_lib.SceneStruct * 1)()
    ms = (_lib.ModelStruct * 1)()
    assert L.dmd_fit_batched(None, 0, sc, ms, 0, None) == 1
    sc[0].n, sc[0].ncols, sc[0].xdtype, sc[0].ldx, sc[0].ldxp = 1000, 30, 0, 1000, 1000
    sc[0].x, sc[0].xp = 0x100, 0x200
    sc[0].opts = _opts(r=40, p=4)          # r > m-1
    ms[0] = _model_struct()
    assert L.dmd_fit_batched(None, 1, sc, ms, 0, None) == 2
    assert L.dmd_graph_launch(None, None) == 1
    assert L.dmd_graph_destroy(None) == 1


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_2502_05339_amd as dmd
    Z = torch.zeros((10, 100), dtype=torch.float32)
    with pytest.raises((RuntimeError, ValueError)):
        dmd.fit(Z, 4)


def test_edit_modes_validation(L):
    """Every rejected argument returns DMD_ERR_ARG before anything is enqueued."""
    from paper_2502_05339_amd import _lib
    m = _model_struct(r=10)

    def edit(**kw):
        e = _lib.EditStruct()
        e.freq_cut = kw.get("freq_cut", 0.01)
        for f in ("weight", "re_scale", "im_scale"):
            getattr(e, f)[0] = getattr(e, f)[1] = 1.0
        for k, v in kw.items():
            if k != "freq_cut":
                getattr(e, k)[1] = v
        return e
    e = edit()
    assert L.dmd_edit_modes(None, ctypes.byref(m), None, 0, 0x1000, 0x2000, 0) == 1
    assert L.dmd_edit_modes(None, ctypes.byref(m), ctypes.byref(e), 0, 0, 0x2000, 0) == 1
    assert L.dmd_edit_modes(None, ctypes.byref(m), ctypes.byref(e), 0, 0x1000, 0, 0) == 1
    assert L.dmd_edit_modes(None, None, ctypes.byref(e), 0, 0x1000, 0x2000, 0) == 1
    for bad in (edit(freq_cut=-0.5), edit(freq_cut=float("nan")), edit(weight=float("inf")),
                edit(re_shift=float("nan")), edit(im_scale=float("-inf"))):
        assert L.dmd_edit_modes(None, ctypes.byref(m), ctypes.byref(bad), 0, 0x1000, 0x2000, 0) == 1
    m.dt = 0.0
    assert L.dmd_edit_modes(None, ctypes.byref(m), ctypes.byref(e), 0, 0x1000, 0x2000, 0) == 1
    m.dt = float("inf")
    assert L.dmd_edit_modes(None, ctypes.byref(m), ctypes.byref(e), 0, 0x1000, 0x2000, 0) == 1


def test_rollout_validation(L):
    """Shape, mode and workspace errors of the forced roll-out, before any GPU work."""
    m = _model_struct(n=1000, r=10)
    nb = ctypes.c_size_t(0)
    assert L.dmd_rollout_workspace_size(1000, 10, 5, 1, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.dmd_rollout_workspace_size(1000, 10, 0, 1, ctypes.byref(nb)) == 2
    assert L.dmd_rollout_workspace_size(1000, 10, 5, 7, ctypes.byref(nb)) == 1
    need = nb.value
    big = 1 << 30
    assert L.dmd_rollout(None, ctypes.byref(m), 0, 0, 1000, 0, 1, 0, 1000, 0, 0x1000, big) == 2      # T = 0
    assert L.dmd_rollout(None, ctypes.byref(m), 0, 0x100, 999, 5, 1, 0, 1000, 0, 0x1000, big) == 1   # ldf < N
    assert L.dmd_rollout(None, ctypes.byref(m), 0, 0, 1000, 5, 0, 0x2000, 1000, 0, 0x1000, big) == 1  # FP64 U, FP32 model
    assert L.dmd_rollout(None, ctypes.byref(m), 0, 0, 1000, 5, 1, 0x2000, 999, 0, 0x1000, big) == 1   # ldu < N
    assert L.dmd_rollout(None, ctypes.byref(m), 0, 0, 1000, 5, 9, 0, 1000, 0, 0x1000, big) == 1       # mode
    assert L.dmd_rollout(None, ctypes.byref(m), 0, 0, 1000, 5, 1, 0, 1000, 0, 0x1000, need - 1) == 3  # workspace
    m.dt = 0.0
    assert L.dmd_rollout(None, ctypes.byref(m), 0, 0, 1000, 5, 1, 0, 1000, 0, 0x1000, big) == 1


def test_upsample_and_lowres_validation(L):
    m = _model_struct(n=1000, r=10)
    nb = ctypes.c_size_t(0)
    assert L.dmd_upsample_workspace_size(1000, 10, 4, 1, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.dmd_upsample_workspace_size(1000, 10, 0, 1, ctypes.byref(nb)) == 2
    flags = (ctypes.c_int32 * 10)()
    big = 1 << 30
    assert L.dmd_upsample(None, ctypes.byref(m), 0, 0x100, 1000, 4, flags, 1, 0, 1000, 0, 0x1000, big) == 1   # h0
    assert L.dmd_upsample(None, ctypes.byref(m), 0x100, 0x200, 999, 4, flags, 1, 0, 1000, 0, 0x1000, big) == 1
    assert L.dmd_upsample(None, ctypes.byref(m), 0x100, 0x200, 1000, 4, None, 1, 0, 1000, 0, 0x1000, big) == 1
    assert L.dmd_upsample(None, ctypes.byref(m), 0x100, 0x200, 1000, 0, flags, 1, 0, 1000, 0, 0x1000, big) == 2
    assert L.dmd_upsample(None, ctypes.byref(m), 0x100, 0x200, 1000, 4, flags, 1, 0, 1000, 0, 0x1000, 16) == 3
    # low-res projection: shapes, dtype, leading dimensions
    P = L.dmd_lowres_project
    assert P(None, 0, 0x100, 200, 0x200, 50, 0x300, 200, 1, 2, 1, 10, 10, 3) == 2           # 10 % 3
    assert P(None, 0, 0x100, 200, 0x200, 50, 0x300, 200, 1, 2, 4, 10, 10, 3) == 2
    assert P(None, 5, 0x100, 200, 0x200, 50, 0x300, 200, 1, 2, 1, 10, 10, 2) == 1           # dtype
    assert P(None, 0, 0x100, 199, 0x200, 50, 0x300, 200, 1, 2, 1, 10, 10, 2) == 1           # ldh < N
    assert P(None, 0, 0x100, 200, 0x200, 49, 0x300, 200, 1, 2, 1, 10, 10, 2) == 1           # ldl < M
    assert P(None, 0, 0x100, 200, 0x200, 50, 0, 200, 1, 2, 1, 10, 10, 2) == 1               # null x
    assert P(None, 0, 0x100, 200, 0x200, 50, 0x300, 200, 0, 2, 1, 10, 10, 2) == 0           # no frames: no-op


def test_fit_workspace_covers_every_valid_ldphi(L):
    """The size query has no model, so it must cover the largest ldphi the header allows
    (192), in both snapshot layouts: a fit into a workspace of exactly the queried size
    passes the workspace checks (it then stops at the HIP runtime, which has no GPU here)."""
    for precision, dt, ncols in (("mixed", 0, 199), ("fp64", 1, 199), ("fp64_exact", 1, 64)):
        o = _opts(150 if precision != "fp64_exact" else 16, 10 if precision != "fp64_exact" else 0, 2, precision)
        n = 4096
        st, need = _ws_size(L, n, ncols, dt, o)
        assert st == 0
        for ldphi in (160 if precision != "fp64_exact" else 32, 192):
            m = _model_struct(n=n, r=o.r, dtype=dt, ldphi=ldphi)
            # separate X and X' (not the shifted view of one buffer)
            code = L.dmd_fit(None, 0x100000, 0x90000000, n, ncols, n, n, dt, ctypes.byref(o), 0x1000, need,
                             ctypes.byref(m))
            assert code not in (1, 2, 3), (precision, ldphi, code)
            assert L.dmd_fit(None, 0x100000, 0x90000000, n, ncols, n, n, dt, ctypes.byref(o), 0x1000, need - 1,
                             ctypes.byref(m)) == 3


def test_status_word_arguments(L):
    st = ctypes.c_int32(0)
    assert L.dmd_status_word(None, None, ctypes.byref(st)) == 1
    assert L.dmd_status_word(None, 0x1000, None) == 1


def _model_file(path, n=5, r=3, dtype=0, dt=0.5, corrupt=None):
    """A model file written byte by byte from the format the header documents."""
    import struct
    import numpy as np
    rng = np.random.default_rng(7)
    lam = rng.standard_normal(2 * r)
    b = rng.standard_normal(2 * r)
    sigma = np.abs(rng.standard_normal(r))
    kind = np.array([1, 2, 0][:r] + [0] * max(0, r - 3), dtype=np.int32)
    phi = rng.standard_normal((n, r)).astype(np.float64 if dtype == 1 else np.float32)
    payload = lam.tobytes() + b.tobytes() + sigma.tobytes() + kind.tobytes() + phi.tobytes()
    h = 1469598103934665603
    for c in payload:
        h = ((h ^ c) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    if corrupt == "hash":
        h ^= 1
    magic = b"DMDMODEL" if corrupt != "magic" else b"DMDMODEX"
    version = 1 if corrupt != "version" else 2
    header = magic + struct.pack("<IIqiidQQII", version, 64, n, r, dtype, dt, len(payload), h, 2, 0)
    assert len(header) == 64
    data = header + payload
    if corrupt == "truncated":
        data = data[:-3]
    if corrupt == "trailing":
        data = data + b"\0"
    with open(path, "wb") as f:
        f.write(data)
    return lam, b, sigma, kind, phi


def test_model_file_header(L, tmp_path):
    """dmd_model_file_info reads the documented layout and rejects foreign, damaged,
    truncated and over-long files (host only)."""
    n_, r_, d_, t_ = ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
    args = (ctypes.byref(n_), ctypes.byref(r_), ctypes.byref(d_), ctypes.byref(t_))
    for dtype in (0, 1):
        p = tmp_path / f"ok{dtype}.dmd"
        _model_file(p, n=7, r=3, dtype=dtype, dt=0.25)
        assert L.dmd_model_file_info(str(p).encode(), *args) == 0
        assert (n_.value, r_.value, d_.value, t_.value) == (7, 3, dtype, 0.25)
    for bad in ("hash", "magic", "version", "truncated", "trailing"):
        p = tmp_path / f"{bad}.dmd"
        _model_file(p, corrupt=bad)
        assert L.dmd_model_file_info(str(p).encode(), *args) == 12, bad
    assert L.dmd_model_file_info(str(tmp_path / "missing.dmd").encode(), *args) == 12
    assert L.dmd_model_file_info(None, *args) == 1


def test_model_load_validation(L, tmp_path):
    """A file that does not fit the caller's model is refused before any device copy."""
    p = tmp_path / "m.dmd"
    _model_file(p, n=7, r=3, dtype=0)
    assert L.dmd_model_load(None, str(p).encode(), ctypes.byref(_model_struct(n=8, r=3))) == 2      # N differs
    assert L.dmd_model_load(None, str(p).encode(), ctypes.byref(_model_struct(n=7, r=3, dtype=1))) == 1
    assert L.dmd_model_load(None, str(p).encode(), ctypes.byref(_model_struct(n=7, r=3, ldphi=16))) == 1
    assert L.dmd_model_load(None, str(tmp_path / "none.dmd").encode(), ctypes.byref(_model_struct(n=7))) == 12
    m = _model_struct(n=7)
    m.phi = 0
    assert L.dmd_model_load(None, str(p).encode(), ctypes.byref(m)) == 1
    assert L.dmd_model_save(None, None, str(p).encode()) == 1
