"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (autotuned decomposition, graph replay).

The oracle cannot step a 200^3 or 400^3 grid in seconds, but one time step
moves information by at most 6 cells along each axis (two half steps of the
3-cell stencil per sweep; the three sweeps act axis by axis), so the state of
one cell after s steps depends only on the box of +-6 s cells around it.  The
oracle steps that box (clipped to the grid, so real grid faces keep their
outflow boundary) and its centre cell is compared with the GPU's; box faces
inside the grid are 6 s cells away and cannot reach the centre.  Properties
that hold at any size (planar invariance, batching, the conservation ledger,
the mixed-precision bound) are checked on the whole grid.
"""
import numpy as np
import pytest

from conftest import to_cons
from paper_1206_0919_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def B(torch):
    from paper_1206_0919_amd import binding
    return binding


def bench_state(B, torch, wl, precision=None, prims=None):
    """A handle on the workload as bench.py builds and tunes it."""
    dims = wl["dims"] if isinstance(wl["dims"], list) else [wl["dims"]]
    kind, params = wl["eos"]
    eos = (B.EOS_BAG, params) if kind == "bag" else None
    if precision is None:
        precision = B.FP32_MIXED if wl["precision"] == "fp32" else B.FP64
    prims = prims if prims is not None else wl["init"]()
    if not isinstance(prims, list):
        prims = [prims]
    s = B.Shasta(dims, wl["dx"], precision=precision, eos=eos)
    for k, pr in enumerate(prims):
        s.write_primitive(k, *[torch.from_numpy(a) for a in pr.as_tuple()])
    dt = wl["lam"] * wl["dx"]
    s.step(dt, 2)              # clocks up, as bench.py does before tuning
    return s, prims, dt


def sample_cells(shape, n_random, seed):
    """Corners, face centres, edges and random cells (x, y, z)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    cells = {(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)}
    cells |= {(nx // 2, ny // 2, 0), (nx // 2, ny // 2, nz - 1), (0, ny // 2, nz // 2),
              (nx - 1, ny // 2, nz // 2), (nx // 2, 0, nz // 2), (nx // 2, ny - 1, nz // 2),
              (1, 2, nz // 3), (nx - 2, ny - 3, 2 * nz // 3), (nx // 2, ny // 2, nz // 2)}
    while len(cells) < 17 + n_random:
        cells.add((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    return sorted(cells)


def oracle_cells(orc, U0, cells, steps, k0, lam):
    """The state of each cell after `steps` steps, from the oracle stepping
    the box of +-6 steps cells around it (clipped to the grid)."""
    r = 6 * steps
    nz, ny, nx = U0[0].shape
    out = []
    for (x, y, z) in cells:
        zs = slice(max(0, z - r), min(nz, z + r + 1))
        ys = slice(max(0, y - r), min(ny, y + r + 1))
        xs = slice(max(0, x - r), min(nx, x + r + 1))
        sub = [np.ascontiguousarray(a[zs, ys, xs]) for a in U0]
        orc.run(sub, lam, steps, k0=k0)
        out.append([a[z - zs.start, y - ys.start, x - xs.start] for a in sub])
    return np.array(out)   # (cells, 5)


def compare_cells(got_fields, ref, cells, label):
    """Relative error per field against the largest |value| of the field on the
    whole GPU grid (for the momenta: of any component)."""
    got = np.array([[f[z, y, x] for f in got_fields] for (x, y, z) in cells])
    Mmax = max(np.abs(got_fields[q]).max() for q in (1, 2, 3))
    worst = 0.0
    for q in range(5):
        den = Mmax if q in (1, 2, 3) else np.abs(got_fields[q]).max()
        err = np.abs(got[:, q] - ref[:, q]).max() / max(den, 1e-300)
        worst = max(worst, err)
    print(label, "sampled cells", len(cells), "max rel error", worst)
    return worst


def test_hotspots200_fp64_full_grid_guard_regime(B, torch, orc):
    # The metric's workload: 200^3 FP64, autotuned, graph replay, 60 steps
    # from the initial state: every cell against the oracle.  From about step
    # 30 on the recovery's admissibility guard (the relativistic correction of
    # Sec. 3) clamps recoveries in the rarefied regions; the guard counts,
    # sums, ledger and largest Courant number match the oracle's too.
    wl = inputs.workload("hotspots200")
    prim = wl["init"]()
    s, _, dt = bench_state(B, torch, wl, prims=prim)
    s.autotune(dt, 2)
    s.write_primitive(0, *[torch.from_numpy(a) for a in prim.as_tuple()])
    s.set_step_index(0)
    steps = 60
    s.step(dt, steps)
    red = s.reduce(0)
    got = [a.cpu().numpy() for a in s.read_conserved(0)]
    s.close()
    U = to_cons(orc, prim)
    ledger, maxeps, cnt = orc.run(U, wl["lam"], steps)
    Mmax = max(np.abs(U[q]).max() for q in (1, 2, 3))
    errs = []
    for q in range(5):
        den = Mmax if q in (1, 2, 3) else np.abs(U[q]).max()
        errs.append(float(np.abs(got[q] - U[q]).max() / den))
    print("hotspots200 60 steps rel errors", errs, "oracle counters", cnt,
          "GPU", red["clamp"], red["floor"], red["noconv"])
    assert max(errs) <= TOL64
    assert cnt[0] > 0
    assert [red["clamp"], red["floor"], red["noconv"]] == cnt[:3]
    assert red["max_eps"] == pytest.approx(maxeps, rel=1e-12, abs=0)
    scale = max(float(np.abs(a).sum()) for a in U)
    sums = np.array([orc.total(a) for a in U])
    np.testing.assert_allclose(red["sums"], sums, rtol=0, atol=1e-12 * scale)
    # 60 steps: the waves have not reached the faces, the outflow is rounding
    np.testing.assert_allclose(red["outflow"], ledger, rtol=1e-11, atol=1e-13 * scale)


def test_hotspots200_conservation_at_full_size(B, torch):
    # sum U(t) - sum U(0) + net outflow = 0 over the whole 200^3 grid
    wl = inputs.workload("hotspots200")
    s, _, dt = bench_state(B, torch, wl)
    s.autotune(dt, 2)
    red0 = s.reduce()
    sums0 = np.array(red0["sums"])
    out0 = np.array(red0["outflow"])
    s.step(dt, 25)
    red = s.reduce()
    resid = np.array(red["sums"]) - sums0 + (np.array(red["outflow"]) - out0)
    scale = np.abs(sums0).max()
    print("ledger residual", resid / scale)
    assert np.abs(resid).max() <= 1e-12 * scale
    assert red["nonfinite"] == 0


def test_shock256_planar_fp64_and_mixed_bound(B, torch, orc):
    # 256^3 planar shock tube, 100 steps: FP64 equals the oracle on 256 x 4 x 4
    # (planar invariance), and the FP32-mixed run of the benchmark stays within
    # the mixed-precision bound of it on the whole grid
    wl = inputs.workload("shock256_mixed")
    prim = wl["init"]()
    s64, _, dt = bench_state(B, torch, wl, precision=B.FP64, prims=prim)
    s64.autotune(dt, 2)
    s64.write_primitive(0, *[torch.from_numpy(a) for a in prim.as_tuple()])
    s64.set_step_index(0)
    s64.step(dt, wl["steps"])
    got64 = [a.cpu().numpy() for a in s64.read_conserved(0)]
    s64.close()
    U = to_cons(orc, inputs.shock_tube((256, 4, 4), wl["dx"]))
    orc.run(U, wl["lam"], wl["steps"])
    Mmax = np.abs(U[1]).max()
    for q in range(5):
        ref = U[q][0, 0, :]
        den = Mmax if q in (1, 2, 3) else np.abs(ref).max()
        if den == 0.0:
            assert np.all(got64[q] == 0.0), q
            continue
        err = np.abs(got64[q] - ref[None, None, :]).max() / den
        print("shock256 FP64 field", q, "rel error", err)
        assert err <= TOL64
    s32, _, _ = bench_state(B, torch, wl, prims=prim)
    s32.autotune(dt, 2)
    s32.write_primitive(0, *[torch.from_numpy(a) for a in prim.as_tuple()])
    s32.set_step_index(0)
    s32.step(dt, wl["steps"])
    got32 = [a.cpu().numpy() for a in s32.read_conserved(0)]
    for q in (0, 1, 4):
        err = np.abs(got32[q] - got64[q]).max() / np.abs(got64[q]).max()
        l1 = np.abs(got32[q] - got64[q]).sum() / np.abs(got64[q]).sum()
        print("shock256 mixed field", q, "max rel", err, "L1", l1)
        assert err <= 2e-4 and l1 <= 2e-5


def test_batch96_equals_single_events_and_oracle(B, torch, orc):
    # 96 events batched (FP32 fields + FP64 recovery, autotuned) against the
    # same events run alone, bitwise, and three whole events against the
    # oracle after 10 steps (FP64 from the FP32-rounded initial state)
    wl = inputs.workload("batch96")
    prims = wl["init"]()
    s, _, dt = bench_state(B, torch, wl, prims=prims)
    s.autotune(dt, 2)
    for k, pr in enumerate(prims):
        s.write_primitive(k, *[torch.from_numpy(a) for a in pr.as_tuple()])
    s.set_step_index(3)
    steps = 10
    s.step(dt, steps)
    sizes = [p.e.size for p in prims]
    picks = [int(np.argmax(sizes)), int(np.argmin(sizes)), 37]
    for k in picks:
        pr = prims[k]
        nz, ny, nx = pr.e.shape
        one = B.Shasta([(nx, ny, nz)], wl["dx"], precision=B.FP32_MIXED)
        one.write_primitive(0, *[torch.from_numpy(a) for a in pr.as_tuple()])
        one.set_step_index(3)
        one.step(dt, steps)
        a = [x.cpu().numpy() for x in s.read_conserved(k)]
        b = [x.cpu().numpy() for x in one.read_conserved(0)]
        for q in range(5):
            assert np.array_equal(a[q], b[q]), (k, q)
        one.close()
        # oracle, FP64 from the FP32-rounded initial conserved state, whole
        # event; bound of the mixed mode over 10 steps (FP32 rounding of about
        # 20 operations per field and half step: 10 x 6 x 20 x 6e-8 = 7e-5)
        U = [x.astype(np.float32).astype(np.float64) for x in to_cons(orc, pr)]
        orc.run(U, wl["lam"], steps, k0=3)
        Mmax = max(np.abs(U[q]).max() for q in (1, 2, 3))
        err = max(np.abs(a[q] - U[q]).max() / (Mmax if q in (1, 2, 3) else np.abs(U[q]).max())
                  for q in range(5))
        l1 = max(np.abs(a[q] - U[q]).sum() / np.abs(U[q]).sum() for q in (0, 4))
        print(f"batch96 event {k} {pr.e.shape[::-1]} 10 steps vs oracle: max rel {err}, L1 {l1}")
        assert err <= 1e-4 and l1 <= 1e-5


def test_bag400_crop_fp64_vs_oracle(B, torch, orc_bag):
    # The bag-model workload's central 100^3 crop (dx 0.1 fm, the longitudinal
    # flow and hot spots of the 400^3 state) as an event of its own, FP64,
    # 30 steps: every cell against the oracle, and the state visits the three
    # branches of the EOS
    wl = inputs.workload("bag400")
    full = wl["init"]()
    c = slice(150, 250)
    prim = inputs.Primitive(*[np.ascontiguousarray(a[c, c, c]) for a in full.as_tuple()])
    del full
    Bc, e_H = wl["eos"][1]
    s = B.Shasta([(100, 100, 100)], wl["dx"], eos=(B.EOS_BAG, (Bc, e_H)))
    s.write_primitive(0, *[torch.from_numpy(a) for a in prim.as_tuple()])
    dt = wl["lam"] * wl["dx"]
    s.step(dt, 30)
    got = [a.cpu().numpy() for a in s.read_conserved(0)]
    U = to_cons(orc_bag, prim)
    orc_bag.run(U, wl["lam"], 30)
    Mmax = max(np.abs(U[q]).max() for q in (1, 2, 3))
    errs = [float(np.abs(got[q] - U[q]).max() / (Mmax if q in (1, 2, 3) else np.abs(U[q]).max()))
            for q in range(5)]
    print("bag400 crop 30 steps rel errors", errs)
    assert max(errs) <= TOL64
    P = orc_bag.cons_to_prim(*U)
    eQ = e_H + 4 * Bc
    assert (P["e"] < e_H).any() and ((P["e"] > e_H) & (P["e"] < eQ)).any() and (P["e"] > eQ).any()


def test_bag400_sampled_cells_and_mixed_bound(B, torch, orc_bag):
    # 400^3, bag EOS, 10 steps: FP64 sampled cells against the oracle, and the
    # FP32-mixed run of the benchmark (autotuned) within the mixed-precision
    # bound of FP64 on the whole grid
    wl = inputs.workload("bag400")
    prim = wl["init"]()
    steps = 10
    s64, _, dt = bench_state(B, torch, wl, precision=B.FP64, prims=prim)
    s64.write_primitive(0, *[torch.from_numpy(a) for a in prim.as_tuple()])
    s64.set_step_index(0)
    s64.step(dt, steps)
    got64 = s64.read_conserved(0)
    s64.close()
    U0 = to_cons(orc_bag, prim)
    cells = sample_cells(prim.e.shape, 0, seed=5)[::2] + [(201, 188, 203), (95, 300, 140)]
    ref = oracle_cells(orc_bag, U0, cells, steps, 0, wl["lam"])
    del U0
    got64_np = [a.cpu().numpy() for a in got64]
    assert compare_cells(got64_np, ref, cells, "bag400 FP64 10 steps") <= TOL64
    del got64_np
    s32, _, _ = bench_state(B, torch, wl, prims=prim)
    s32.autotune(dt, 2)
    s32.write_primitive(0, *[torch.from_numpy(a) for a in prim.as_tuple()])
    s32.set_step_index(0)
    s32.step(dt, steps)
    got32 = s32.read_conserved(0)
    Mmax = max(got64[q].abs().max().item() for q in (1, 2, 3))
    for q in range(5):
        d = (got32[q] - got64[q]).abs()
        err = d.max().item() / (Mmax if q in (1, 2, 3) else got64[q].abs().max().item())
        l1 = (d.sum() / got64[q].abs().sum()).item()
        print("bag400 mixed field", q, "max rel", err, "L1", l1)
        assert err <= 1e-4 and (q in (1, 2) or l1 <= 1e-5)


@pytest.mark.parametrize("precision,dims", [(0, (1023, 1024, 256)), (1, (1023, 1024, 512))])
def test_largest_event_sampled_cells(B, torch, orc, precision, dims):
    # the largest event shasta_create accepts: a field array just below 2^31
    # bytes (the kernels address fields with 32-bit byte offsets); cells near
    # the last bytes of the arrays against the oracle after one step
    nx, ny, nz = dims
    esize = 8 if precision == 0 else 4
    assert nx * ny * nz * esize < 2 ** 31 <= (nx + 1) * ny * nz * esize
    s = B.Shasta([dims], 0.2, precision=precision)
    X, Y, Z = (torch.arange(n, dtype=torch.float64, device="cuda") for n in (nx, ny, nz))
    e = 1.0 + 0.5 * torch.sin(0.05 * X)[None, None, :] * torch.cos(0.07 * Y)[None, :, None] \
        * torch.sin(0.03 * Z + 0.4)[:, None, None]
    zero = torch.zeros_like(e)
    vz = 0.3 * torch.tanh(0.01 * (Z - nz / 2))[:, None, None].expand_as(e).contiguous()
    s.write_primitive(0, e, zero, zero, vz, 0.15 * e)
    del zero
    s.set_step_index(2)
    s.step(0.08, 1)
    cells = [(nx - 1, ny - 1, nz - 1), (nx - 2, ny - 1, nz - 1), (nx - 1, ny - 7, nz - 3),
             (0, ny - 1, nz - 1), (nx // 2, ny - 1, nz - 2), (nx - 1, 0, nz - 1),
             (nx // 3, ny // 2, nz - 1), (7, 9, nz // 2), (nx - 1, ny - 1, 0)]
    got = []
    for q in range(5):
        f = s.read_field(0, q)
        got.append([f[z, y, x].item() for (x, y, z) in cells])
        del f
    got = np.array(got).T
    # oracle: the +-6 box of each cell, from the same primitives (rounded to
    # the field precision for FP32)
    r = 6
    ref = []
    for (x, y, z) in cells:
        zs = slice(max(0, z - r), min(nz, z + r + 1))
        ys = slice(max(0, y - r), min(ny, y + r + 1))
        xs = slice(max(0, x - r), min(nx, x + r + 1))
        pe = e[zs, ys, xs].cpu().numpy()
        pvz = vz[zs, ys, xs].cpu().numpy()
        z0 = np.zeros_like(pe)
        prim = inputs.Primitive(np.ascontiguousarray(pe), z0, z0.copy(),
                                np.ascontiguousarray(pvz), 0.15 * pe)
        U = to_cons(orc, prim)
        if precision == 1:
            U = [a.astype(np.float32).astype(np.float64) for a in U]
        orc.run(U, 0.4, 1, k0=2)
        ref.append([a[z - zs.start, y - ys.start, x - xs.start] for a in U])
    ref = np.array(ref)
    scale = [1.5, 1.0, 1.0, 1.0, 0.3]   # |E| and |R| <= 1.5 (R ~ 0.15 E gamma), |M| < 1
    err = max(np.abs(got[:, q] - ref[:, q]).max() / scale[q] for q in range(5))
    print("largest event, precision", precision, "max rel error", err)
    assert err <= (TOL64 if precision == 0 else 2e-5)
