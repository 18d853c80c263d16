"""GPU parity of the double-layer operator under AIMx (Sec. III-B, eq. KAIMx)
against oracle/dlp.py, through the C ABI: the static near values and their
precorrection on the near list, and the matvec with several right-hand
sides at several wavenumbers, including the full-size box array on sampled
rows."""
import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx, dlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU machines skip the module
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("make", [I.sphere_small, I.small_box_array])
def test_near_values_and_matvec(make):
    w = make()
    ks = [float(w.k[0]), 8.5]
    print(f"[gpu] double layer {make.__name__}", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    d = dlp.DlpOracle(o)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, ks,
                     max_rhs=3)
    rows, cols = o.near_list()
    near, corr = p.dlp_values()
    ref_near = dlp.static_near(o.V, o.T, rows, cols)
    ref_corr = d.correction_values(rows, cols)
    assert np.max(np.abs(near - ref_near)) <= 1e-13 * np.max(np.abs(ref_near))
    assert np.max(np.abs(corr - ref_corr)) <= 1e-13 * np.max(np.abs(ref_corr))
    x = I.complex_gaussian(o.N, 41, nrhs=3)
    freq = [0, 1, 0]
    y = p.matvec_dlp(torch.from_numpy(x).cuda(), freq_idx=freq).cpu().numpy()
    for r in range(3):
        assert rel(y[r], d.matvec(x[r], ks[freq[r]])) <= 1e-10, r
    y1 = p.matvec_dlp(torch.from_numpy(x[1]).cuda(), freq_idx=[1]).cpu().numpy()
    assert rel(y1, d.matvec(x[1], ks[1])) <= 1e-10
    p.close()


def test_full_size_box_array_sampled_rows():
    w = I.box_array_large()
    print("[gpu] double layer, full-size box array", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     precisions=("c128",))
    x = I.complex_gaussian(o.N, 43)
    rows = np.sort(np.random.default_rng(44).choice(o.N, 16, replace=False))
    ref = dlp.DlpOracle(o).matvec_rows(x, float(w.k[0]), rows)
    y = p.matvec_dlp(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y[rows], ref) <= 1e-10
    p.close()


def test_needs_the_mesh(tmp_path):
    w = I.sphere_tiny()
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
    path = str(tmp_path / "plan.bin")
    p.save(path)
    q = binding.Plan.load(path)
    x = torch.zeros(q.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.AimError) as e:
        q.matvec_dlp(x)
    assert e.value.status == 8
    q.close()
    p.close()
