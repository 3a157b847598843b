"""The C-ABI library loads and exports every symbol include/shasta.h
declares; host-side argument validation works without touching a GPU (every
call below returns before its first HIP call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shasta.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shasta_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def b():
    from paper_1206_0919_amd import binding
    return binding


def test_header_declares_the_boundary():
    names = declared()
    for n in ("shasta_create", "shasta_workspace_bytes", "shasta_bind_workspace",
              "shasta_set_eos", "shasta_write_primitive", "shasta_write_conserved",
              "shasta_set_step_index", "shasta_step", "shasta_read_field",
              "shasta_reduce", "shasta_destroy", "shasta_last_error",
              "shasta_status_str"):
        assert n in names


def test_library_exports_every_declared_symbol(b):
    lib = ctypes.CDLL(b.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert set(declared()) == set(b.EXPORTS)


def _create(b, n, dims, dx=0.2, prec=0, bc=0):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int32 * len(dims))(*dims)
    st = b.shasta_create(ctypes.byref(h), n, arr, dx, prec, bc, None)
    return st, h


def test_create_validation(b):
    assert _create(b, 0, [4, 4, 4])[0] == b.EINVAL
    assert _create(b, 1, [4, 0, 4])[0] == b.EINVAL
    assert _create(b, 1, [4, 4, 4], dx=0.0)[0] == b.EINVAL
    assert _create(b, 1, [4, 4, 4], dx=float("nan"))[0] == b.EINVAL
    assert _create(b, 1, [4, 4, 4], prec=2)[0] == b.EINVAL
    assert _create(b, 1, [4, 4, 4], bc=1)[0] == b.EINVAL
    assert _create(b, 1, [2048, 2048, 1024])[0] == b.EINVAL  # > 2^31 cells
    # one field array must stay below 2^31 bytes (32-bit buffer offsets)
    assert _create(b, 1, [1024, 1024, 257])[0] == b.EINVAL            # FP64: 2.06 GiB
    assert _create(b, 1, [1024, 1024, 513], prec=1)[0] == b.EINVAL    # FP32: 2.004 GiB
    st, h = _create(b, 2, [4, 5, 6, 48, 64, 96], prec=1)
    assert st == b.OK
    nb = ctypes.c_size_t()
    assert b.shasta_workspace_bytes(h, ctypes.byref(nb)) == b.OK
    # two FP32 buffers of 5 fields per event, 64-element pitch
    assert nb.value >= 4 * 5 * 2 * (128 + 48 * 64 * 96)
    assert b.shasta_destroy(h) == b.OK


def test_state_and_eos_validation(b):
    st, h = _create(b, 1, [8, 8, 8])
    assert st == b.OK
    # step before a workspace is bound (both forms)
    assert b.shasta_step(h, 0.08, 1) == b.ESTATE
    assert b"workspace" in b.shasta_last_error(h)
    assert b.shasta_step_noalloc(h, 0.08, 1) == b.ESTATE
    assert b.shasta_step_noalloc(h, 0.1, 1) == b.EINVAL
    assert b.shasta_step_noalloc(h, 0.08, -1) == b.EINVAL
    # dt/dx must be in (0, 1/2)
    assert b.shasta_step(h, 0.1, 1) == b.EINVAL
    assert b.shasta_step(h, -0.01, 1) == b.EINVAL
    assert b.shasta_step(h, 0.08, -1) == b.EINVAL
    p = (ctypes.c_double * 2)(0.4, 0.1)
    assert b.shasta_set_eos(h, 1, p, 2) == b.OK
    assert b.shasta_set_eos(h, 1, p, 1) == b.EINVAL
    bad = (ctypes.c_double * 2)(-1.0, 0.1)
    assert b.shasta_set_eos(h, 1, bad, 2) == b.EINVAL
    assert b.shasta_set_eos(h, 7, None, 0) == b.EINVAL
    assert b.shasta_set_eos(h, 0, None, 0) == b.OK
    # tabled EOS: {e_0..e_m-1, p_0..p_m-1}
    def table(vals):
        return (ctypes.c_double * len(vals))(*vals), len(vals)
    good = [0.0, 1.0, 2.0, 0.0, 0.3, 0.5]
    assert b.shasta_set_eos(h, 2, *table(good)) == b.OK
    for bad_t in ([0.0, 1.0, 0.0], [0.1, 1.0, 0.0, 0.3],          # odd n, e_0 != 0
                  [0.0, 1.0, 1.0, 0.0, 0.3, 0.5],                  # e not increasing
                  [0.0, 1.0, 2.0, 0.0, 1.5, 1.6],                  # slope > 1
                  [0.0, 1.0, 2.0, 0.0, 0.3, 0.2],                  # slope < 0
                  [0.0, 1.0, -0.1, 0.2], [0.0, float("nan"), 0.0, 0.1]):
        assert b.shasta_set_eos(h, 2, *table(bad_t)) == b.EINVAL, bad_t
    # baryon-dependent EOS: {cs2, mass}
    for bad_b in ([0.0, 0.9], [1.2, 0.9], [0.3, -1.0], [0.3, float("inf")], [0.3]):
        assert b.shasta_set_eos(h, 3, *table(bad_b)) == b.EINVAL, bad_b
    assert b.shasta_set_eos(h, 3, *table([1.0 / 3.0, 0.938])) == b.OK
    # {cs2, mass, iterations}: an integer cap of the root solve in [1, 64]
    for bad_it in (0.0, 65.0, 2.5, -1.0, float("nan")):
        assert b.shasta_set_eos(h, 3, *table([1.0 / 3.0, 0.938, bad_it])) == b.EINVAL, bad_it
    for it in (1.0, 16.0, 64.0):
        assert b.shasta_set_eos(h, 3, *table([1.0 / 3.0, 0.938, it])) == b.OK
    big = [float(k) for k in range(1025)] + [k / 3.0 for k in range(1025)]
    assert b.shasta_set_eos(h, 2, *table(big)) == b.EINVAL           # more than 1024 nodes
    assert b.shasta_set_eos(h, 0, None, 0) == b.OK
    assert b.shasta_set_step_index(h, -3) == b.EINVAL
    assert b.shasta_set_tiles(h, 1, 8, 16) == b.EINVAL   # segment < 16
    assert b.shasta_set_tiles(h, 2, 32, 48) == b.EINVAL  # lanes not 16/32/64
    assert b.shasta_set_tiles(h, 3, 32, 16) == b.EINVAL
    assert b.shasta_set_tiles(h, 1, 32, 16) == b.OK
    assert b.shasta_set_tiles(h, 2, 32, 1) == b.OK      # flattened columns
    assert b.shasta_set_tiles(h, 2, 32, 2) == b.EINVAL
    for bad_diff in (-0.1, 1.5, float("nan"), float("inf")):
        assert b.shasta_set_antidiffusion(h, bad_diff) == b.EINVAL
    for diff in (0.0, 0.5, 1.0):
        assert b.shasta_set_antidiffusion(h, diff) == b.OK
    out = (ctypes.c_double * 12)()
    cnt = (ctypes.c_int64 * 4)()
    assert b.shasta_reduce(h, 1, out, cnt) == b.EINVAL
    assert b.shasta_reduce(h, 0, out, cnt) == b.ESTATE
    assert b.shasta_read_field(h, 0, 11, None) == b.EINVAL
    assert b.shasta_destroy(h) == b.OK
    assert b.shasta_status_str(b.ENONFINITE) == b"non-finite value in the fields"
    assert b.shasta_status_str(b.ENOCONVERGE) == b"recovery did not converge"
    assert b.shasta_forget_tuning() == b.OK


def test_march_copy_validation(b):
    """Every bad argument is refused on the host, before any launch."""
    p = ctypes.c_void_p(4096)   # never dereferenced: each call below is refused
    n = 8 * 8 * 8
    ok = dict(nx=8, ny=8, nz=8, pitch=n, axis=1, seg=4, prec=0)

    def call(src=p, dst=p, **kw):
        a = dict(ok, **kw)
        return b.shasta_march_copy(src, dst, a["nx"], a["ny"], a["nz"], a["pitch"], a["axis"],
                                   a["seg"], a["prec"], None)

    assert call(src=None) == b.EINVAL
    assert call(dst=None) == b.EINVAL
    assert call(nx=0) == b.EINVAL
    assert call(nz=-1) == b.EINVAL
    assert call(axis=0) == b.EINVAL      # x has no march
    assert call(axis=3) == b.EINVAL
    assert call(seg=0) == b.EINVAL
    assert call(prec=2) == b.EINVAL
    assert call(pitch=n - 1) == b.EINVAL
    # one field array below 2^31 bytes
    assert call(nx=1024, ny=1024, nz=257, pitch=1024 * 1024 * 257) == b.EINVAL
    assert call(nx=1024, ny=1024, nz=513, pitch=1024 * 1024 * 513, prec=1) == b.EINVAL


def test_copy_bindings_check_their_buffers(b):
    # host tensors, short buffers and a wrong element type are refused before
    # any call reaches the library
    import torch
    x = torch.zeros(64, dtype=torch.float64)
    with pytest.raises(ValueError):
        b.stream_copy(x, x, 64, None)
    with pytest.raises(ValueError):
        b.march_copy(x, x, (2, 2, 2), 8, 1, 4, b.FP64, None)
    with pytest.raises(ValueError):
        b.march_copy(x.float(), x.float(), (2, 2, 2), 8, 1, 4, b.FP64, None)
