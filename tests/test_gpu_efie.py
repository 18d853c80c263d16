"""GPU parity of the RWG EFIE under AIMx (Sec. II-A, eq. EFIEdis; Sec. II-B,
eq. LAIMx) against oracle/efie.py, through the C ABI: the RWG numbering and
near list (exact), C_A and C_phi on it, and the product with several
right-hand sides at several wavenumbers -- on a closed sphere, a ragged
third-order box array, an open hemisphere (boundary edges carry no
function) and, on sampled rows, an 81,920-triangle sphere."""
import math

import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx, efie

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU machines skip the module
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402

TOL_C = 1e-12    # static values: closed forms on both sides, fp64
TOL_Y = 1e-10    # products: FFT convolution in fp64 on both sides


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def hemisphere(level=3, radius=0.5):
    V, T = I.icosphere(level, radius)
    cz = V[T].mean(axis=1)[:, 2]
    T = T[cz > 0.0]
    used, inv = np.unique(T.ravel(), return_inverse=True)
    return np.ascontiguousarray(V[used]), inv.reshape(T.shape).astype(np.int32)


def setup(V, T, order, dims, h, tau, ks, max_rhs=3):
    o = aimx.AimOracle(V, T, order, dims, h, tau)
    e = efie.EfieOracle(o)
    p = binding.Plan(V, T, order, dims, h, tau, ks, max_rhs=max_rhs, precisions=("c128",))
    return o, e, p


def check_tables(p, e, rows=None):
    t = p.efie_tables()
    assert np.array_equal(t["tri_rwg"], e.rwg.tri_rwg)
    rowptr, col = t["rowptr"], t["col"]
    got_rows = np.repeat(np.arange(e.n), np.diff(rowptr))
    assert np.array_equal(got_rows, e.rows) and np.array_equal(col, e.cols)
    sel = np.ones(e.rows.size, bool) if rows is None else np.isin(e.rows, rows)
    ca, cq = e.correction_values(e.rows[sel], e.cols[sel])
    assert np.max(np.abs(t["ca"][sel] - ca)) <= TOL_C * np.max(np.abs(ca))
    assert np.max(np.abs(t["cphi"][sel] - cq)) <= TOL_C * np.max(np.abs(cq))


def test_closed_sphere_tables_and_products():
    w = I.sphere_tiny(level=2, dims=(16, 16, 16), h=0.1)
    ks = [2 * math.pi, 8.5]
    print("[gpu] EFIE sphere-320", flush=True)
    o, e, p = setup(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, ks)
    info = p.efie_setup()
    assert info["n_rwg"] == 3 * o.N // 2 == e.n
    check_tables(p, e)
    x = I.complex_gaussian(e.n, 51, nrhs=3)
    freq = [0, 1, 0]
    y = p.matvec_efie(torch.from_numpy(x).cuda(), freq_idx=freq).cpu().numpy()
    for r in range(3):
        ref = e.matvec(x[r], ks[freq[r]])
        assert np.max(np.abs(y[r] - ref)) <= TOL_Y * np.max(np.abs(ref)), r
    y1 = p.matvec_efie(torch.from_numpy(x[2]).cuda(), freq_idx=[1]).cpu().numpy()
    assert rel(y1, e.matvec(x[2], ks[1])) <= TOL_Y
    p.close()


def test_box_array_third_order_sampled_rows():
    w = I.small_box_array()
    print("[gpu] EFIE small box array", flush=True)
    o, e, p = setup(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
    rows = np.arange(0, e.n, 29)
    check_tables(p, e, rows)
    x = I.complex_gaussian(e.n, 52, nrhs=2)
    y = p.matvec_efie(torch.from_numpy(x).cuda()).cpu().numpy()
    for r in range(2):
        ref = e.matvec_rows(x[r], float(w.k[0]), rows)
        assert np.max(np.abs(y[r][rows] - ref)) <= TOL_Y * np.max(np.abs(ref)), r
    p.close()


def test_open_surface():
    V, T = hemisphere()
    h = 0.1
    print("[gpu] EFIE open hemisphere", flush=True)
    o, e, p = setup(V, T, 2, (16, 16, 16), h, 2 * h, [2 * math.pi])
    tab = p.efie_tables()
    boundary = int(np.sum(tab["tri_rwg"] < 0))
    assert boundary > 0 and 2 * e.n + boundary == 3 * T.shape[0]
    rows = np.arange(0, e.n, 15)
    check_tables(p, e, rows)
    x = I.complex_gaussian(e.n, 53)
    y = p.matvec_efie(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = e.matvec_rows(x, 2 * math.pi, rows)
    assert np.max(np.abs(y[rows] - ref)) <= TOL_Y * np.max(np.abs(ref))
    p.close()


def test_large_sphere_sampled_rows():
    w = I.efie_sphere()
    print(f"[gpu] EFIE {w.name}, sampled rows", flush=True)
    o, e, p = setup(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                    max_rhs=1)
    rows = np.sort(np.random.default_rng(54).choice(e.n, 12, replace=False))
    x = I.complex_gaussian(e.n, 55)
    y = p.matvec_efie(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = e.matvec_rows(x, float(w.k[0]), rows)
    assert rel(y[rows], ref) <= TOL_Y
    check_tables(p, e, rows[:4])
    p.close()


def test_rejections(tmp_path):
    w = I.sphere_tiny()
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
    path = str(tmp_path / "plan.bin")
    p.save(path)
    q = binding.Plan.load(path)
    with pytest.raises(binding.AimError) as err:
        q.efie_setup()
    assert err.value.status == 8                      # the mesh is not kept by loaded plans
    q.close()
    p.close()
    # an edge shared by three triangles
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1]], dtype=np.float64) * 0.4
    T = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]], dtype=np.int32)
    p = binding.Plan(V, T, 2, (16, 16, 16), 0.1, 0.2, [2 * math.pi])
    with pytest.raises(binding.AimError) as err:
        p.efie_setup()
    assert err.value.status == 2                      # AIM_ERR_GEOMETRY
    p.close()
