"""igb_potential_noalloc (the potential without any device allocation, for callers that cannot allocate)
against igb_potential on the same operator and density: two calls in a row, the second with fewer points,
within the potential bar (1e-12 relative), for the real and the complex kernel; and the size limit."""
import numpy as np
import pytest

from paper_1708_09162_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
igb = pytest.importorskip("paper_1708_09162_amd.igabem")

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("kind", ["laplace", "helmholtz"])
def test_potential_noalloc_matches_potential(kind):
    print(f"[no-alloc] {kind}: torus p=1 m=2 q=4", flush=True)
    kw = dict(p=1, m=2, q=4, leaf_depth=1, eta=1.6, gauss_regular=6)
    if kind == "helmholtz":
        kw.update(kernel=igb.IGB_HELMHOLTZ, wavenumber=2.0)
    op = igb.Operator(igb.Geometry(W.torus_patches()), mode=igb.IGB_H2_ONTHEFLY, device=DEV, **kw)
    rng = np.random.default_rng(3)
    w = rng.standard_normal(op.info.n_dof)
    if kind == "helmholtz":
        w = w + 1j * rng.standard_normal(op.info.n_dof)
    w = torch.tensor(w, device=DEV)
    for npts in (3000, 700):  # two calls in a row, the second smaller
        pts = 4.0 * W.random_directions(npts, npts) + np.array([0.0, 0.0, 1.0])
        ref = op.potential(w, pts).cpu().numpy()
        out = torch.full((npts,), float("nan"), dtype=op.dtype, device=DEV)
        got = op.potential_noalloc(w, pts, out).cpu().numpy()
        assert np.all(np.isfinite(got))
        assert rel(got, ref) <= 1e-12, (npts, rel(got, ref))
    # beyond the scratch capacity: rejected before any GPU work
    cap = (32 << 20) // (16 if kind == "helmholtz" else 8)
    big = torch.zeros((cap + 1, 3), dtype=torch.float64, device=DEV)
    outb = torch.zeros(cap + 1, dtype=op.dtype, device=DEV)
    with pytest.raises(igb.IgbError) as e:
        igb.igb_potential_noalloc(op.h, w, big, outb)
    assert e.value.status == igb.IGB_EINVAL
