"""The step variant that allocates nothing (shasta_step_noalloc), through the
C ABI, against shasta_step: bitwise the same fields and reductions, on two
calls in a row (the second on a smaller grid), and the size limit of its
static scratch."""
import numpy as np
import pytest

from paper_1206_0919_amd import inputs

pytestmark = pytest.mark.gpu

DX, DT = 0.2, 0.08


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


def _prim(dims, seed):
    rng = np.random.default_rng(seed)
    pr = inputs.hotspots(dims, DX, 6, seed=seed)
    v = rng.uniform(-0.3, 0.3, (3,) + pr.e.shape)
    return inputs.Primitive(pr.e, v[0], v[1], v[2], pr.n)


def _state(B, torch, dims, prim, precision):
    s = B.Shasta([dims], DX, precision=precision)
    s.write_primitive(0, *[torch.from_numpy(a) for a in prim.as_tuple()])
    return s


@pytest.mark.parametrize("precision", [0, 1])
def test_step_noalloc_equals_step_on_two_calls(B, torch, precision):
    # first call on a larger ragged grid, second on a smaller one: the
    # second call reuses the scratch the first one left behind
    for dims, steps, k0, seed in (((45, 38, 29), 7, 2, 31), ((17, 13, 11), 5, 0, 32)):
        prim = _prim(dims, seed)
        ref = _state(B, torch, dims, prim, precision)
        got = _state(B, torch, dims, prim, precision)
        ref.set_step_index(k0)
        got.set_step_index(k0)
        ref.step(DT, steps)
        got.step_noalloc(DT, steps)
        assert got.step_index() == ref.step_index() == k0 + steps
        a = [x.cpu().numpy() for x in ref.read_conserved(0)]
        b = [x.cpu().numpy() for x in got.read_conserved(0)]
        for q in range(5):
            assert np.array_equal(a[q], b[q]), (dims, q)
        ra, rb = ref.reduce(), got.reduce()
        for key in ("sums", "outflow", "max_eps", "t", "clamp", "floor", "noconv",
                    "nonfinite", "status"):
            assert ra[key] == rb[key], (dims, key)
        ref.close()
        got.close()


def test_step_noalloc_persistent_launch(B, torch):
    # the persistent launch takes its queue counters from the static scratch
    dims = (40, 36, 30)
    prim = _prim(dims, 33)
    ref = _state(B, torch, dims, prim, 0)
    got = _state(B, torch, dims, prim, 0)
    for s in (ref, got):
        for ax in range(3):
            s.set_persistent(ax, True)
    ref.step(DT, 6)
    got.step_noalloc(DT, 6)
    a = [x.cpu().numpy() for x in ref.read_conserved(0)]
    b = [x.cpu().numpy() for x in got.read_conserved(0)]
    for q in range(5):
        assert np.array_equal(a[q], b[q]), q


def test_step_noalloc_rejects_oversized_scratch(B, torch):
    # one x window per work item on a large grid: more records than the
    # static scratch holds; rejected before anything is launched
    dims = (400, 400, 120)
    s = B.Shasta([dims], DX)
    e = torch.full((dims[2], dims[1], dims[0]), 1.0, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(e)
    s.write_primitive(0, e, z, z, z, 0.1 * e)
    s.set_tiles(0, 1, 0)
    with pytest.raises(B.ShastaError) as exc:
        s.step_noalloc(DT, 1)
    assert exc.value.status == B.EINVAL and "scratch" in str(exc.value)
    assert s.step_index() == 0
    s.step(DT, 1)          # the ordinary step still runs
    assert s.step_index() == 1
