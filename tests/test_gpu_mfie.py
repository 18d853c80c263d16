"""GPU parity of the RWG double-layer operator under AIMx (Sec. III-B, eq.
KAIMx) against oracle/mfie.py, through the C ABI: C_K = K_s,NR - K_s,P and
the Gram entries on the RWG near list, and (K + beta G) x with several
right-hand sides at several wavenumbers -- on a closed sphere (all rows), a
ragged third-order box array, an open hemisphere and, on sampled rows, an
81,920-triangle sphere."""
import math

import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx, efie, mfie

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU machines skip the module
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402

TOL_C = 1e-12    # static values: closed forms on both sides, fp64
TOL_Y = 1e-10    # products: FFT convolution in fp64 on both sides


def hemisphere(level=3, radius=0.5):
    V, T = I.icosphere(level, radius)
    cz = V[T].mean(axis=1)[:, 2]
    T = T[cz > 0.0]
    used, inv = np.unique(T.ravel(), return_inverse=True)
    return np.ascontiguousarray(V[used]), inv.reshape(T.shape).astype(np.int32)


def setup(V, T, order, dims, h, tau, ks, max_rhs=3):
    o = aimx.AimOracle(V, T, order, dims, h, tau)
    m = mfie.MfieOracle(efie.EfieOracle(o))
    p = binding.Plan(V, T, order, dims, h, tau, ks, max_rhs=max_rhs, precisions=("c128",))
    return m, p


def check_values(p, m, rows=None):
    v = p.mfie_values()
    sel = np.ones(m.rows.size, bool) if rows is None else np.isin(m.rows, rows)
    ck = m.correction_values(m.rows[sel], m.cols[sel])
    gr = m.gram(m.rows[sel], m.cols[sel])
    assert np.max(np.abs(v["ck"][sel] - ck)) <= TOL_C * np.max(np.abs(ck))
    assert np.max(np.abs(v["gram"][sel] - gr)) <= TOL_C * np.max(np.abs(gr))


def test_closed_sphere_values_and_products():
    w = I.sphere_tiny(level=2, dims=(16, 16, 16), h=0.1)
    ks = [2 * math.pi, 8.5]
    print("[gpu] RWG double layer, sphere-320", flush=True)
    m, p = setup(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, ks)
    check_values(p, m)
    x = I.complex_gaussian(m.n, 71, nrhs=3)
    freq = [0, 1, 0]
    y = p.matvec_mfie(torch.from_numpy(x).cuda(), freq_idx=freq, gram_coef=0.5).cpu().numpy()
    for r in range(3):
        ref = m.matvec(x[r], ks[freq[r]], 0.5)
        assert np.max(np.abs(y[r] - ref)) <= TOL_Y * np.max(np.abs(ref)), r
    y1 = p.matvec_mfie(torch.from_numpy(x[1]).cuda(), freq_idx=[1]).cpu().numpy()
    ref = m.matvec(x[1], ks[1], 0.0)
    assert np.max(np.abs(y1 - ref)) <= TOL_Y * np.max(np.abs(ref))
    p.close()


def test_box_array_third_order_sampled_rows():
    w = I.small_box_array()
    print("[gpu] RWG double layer, small box array", flush=True)
    m, p = setup(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
    rows = np.arange(0, m.n, 29)
    check_values(p, m, rows)
    x = I.complex_gaussian(m.n, 72, nrhs=2)
    y = p.matvec_mfie(torch.from_numpy(x).cuda(), gram_coef=-0.5).cpu().numpy()
    for r in range(2):
        ref = m.matvec_rows(x[r], float(w.k[0]), rows, -0.5)
        assert np.max(np.abs(y[r][rows] - ref)) <= TOL_Y * np.max(np.abs(ref)), r
    p.close()


def test_open_surface():
    V, T = hemisphere()
    h = 0.1
    print("[gpu] RWG double layer, open hemisphere", flush=True)
    m, p = setup(V, T, 2, (16, 16, 16), h, 2 * h, [2 * math.pi])
    rows = np.arange(0, m.n, 15)
    check_values(p, m, rows)
    x = I.complex_gaussian(m.n, 73)
    y = p.matvec_mfie(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = m.matvec_rows(x, 2 * math.pi, rows)
    assert np.max(np.abs(y[rows] - ref)) <= TOL_Y * np.max(np.abs(ref))
    p.close()


def test_large_sphere_sampled_rows():
    w = I.efie_sphere()
    print(f"[gpu] RWG double layer, {w.name}, sampled rows", flush=True)
    m, p = setup(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                 max_rhs=1)
    rows = np.sort(np.random.default_rng(74).choice(m.n, 12, replace=False))
    x = I.complex_gaussian(m.n, 75)
    y = p.matvec_mfie(torch.from_numpy(x).cuda(), gram_coef=0.5).cpu().numpy()
    ref = m.matvec_rows(x, float(w.k[0]), rows, 0.5)
    assert np.linalg.norm(y[rows] - ref) <= TOL_Y * np.linalg.norm(ref)
    check_values(p, m, rows[:4])
    p.close()


def test_combined_field_operator():
    """eq. CFIEAIMx: Z x + (j/k)(K + beta G) x from one call, against the two
    oracles on sampled rows, several vectors at two wavenumbers."""
    w = I.sphere_tiny(level=2, dims=(16, 16, 16), h=0.1)
    ks = [2 * math.pi, 8.5]
    print("[gpu] combined field, sphere-320", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    e = efie.EfieOracle(o)
    m = mfie.MfieOracle(e)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, ks,
                     max_rhs=3, precisions=("c128",))
    x = I.complex_gaussian(m.n, 76, nrhs=3)
    freq = [1, 0, 1]
    y = p.matvec_cfie(torch.from_numpy(x).cuda(), freq_idx=freq, gram_coef=-0.5).cpu().numpy()
    rows = np.arange(0, m.n, 6)
    for r in range(3):
        k = ks[freq[r]]
        ref = e.matvec_rows(x[r], k, rows) + 1j / k * m.matvec_rows(x[r], k, rows, -0.5)
        assert np.max(np.abs(y[r][rows] - ref)) <= TOL_Y * np.max(np.abs(ref)), r
    # the separate operators' calls agree with the combined one on every row
    xe = torch.from_numpy(x).cuda()
    ye = p.matvec_efie(xe, freq_idx=freq).cpu().numpy()
    ym = p.matvec_mfie(xe, freq_idx=freq, gram_coef=-0.5).cpu().numpy()
    kk = np.array([ks[f] for f in freq])[:, None]
    comb = ye + 1j / kk * ym
    assert np.max(np.abs(y - comb)) <= 1e-13 * np.max(np.abs(comb))
    p.close()


def test_combined_field_large_sphere_sampled_rows():
    """The combined field on the 81,920-triangle sphere (the double layer
    takes its currents from the EFIE's projection): sampled rows against the
    two oracles."""
    w = I.efie_sphere()
    print(f"[gpu] combined field, {w.name}, sampled rows", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    e = efie.EfieOracle(o)
    m = mfie.MfieOracle(e)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=1, precisions=("c128",))
    k = float(w.k[0])
    rows = np.sort(np.random.default_rng(77).choice(m.n, 10, replace=False))
    x = I.complex_gaussian(m.n, 78)
    y = p.matvec_cfie(torch.from_numpy(x).cuda(), gram_coef=-0.5).cpu().numpy()
    ref = e.matvec_rows(x, k, rows) + 1j / k * m.matvec_rows(x, k, rows, -0.5)
    assert np.linalg.norm(y[rows] - ref) <= TOL_Y * np.linalg.norm(ref)
    p.close()


def test_complex64_operators():
    """The three RWG operators in complex64 (tables rounded from the
    complex128 ones, FFTs and gathers in complex64) against the oracles at
    the FP32 bar, several vectors at two wavenumbers."""
    w = I.sphere_tiny(level=2, dims=(16, 16, 16), h=0.1)
    ks = [2 * math.pi, 8.5]
    print("[gpu] RWG operators in complex64, sphere-320", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    e = efie.EfieOracle(o)
    m = mfie.MfieOracle(e)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, ks,
                     max_rhs=3, precisions=("c128", "c64"))
    x = I.complex_gaussian(m.n, 79, nrhs=3)
    xd = torch.from_numpy(x).to(torch.complex64).cuda()
    freq = [0, 1, 1]
    rows = np.arange(0, m.n, 4)
    ye = p.matvec_efie(xd, freq_idx=freq, prec="c64").cpu().numpy()
    ym = p.matvec_mfie(xd, freq_idx=freq, gram_coef=-0.5, prec="c64").cpu().numpy()
    yc = p.matvec_cfie(xd, freq_idx=freq, gram_coef=-0.5, prec="c64").cpu().numpy()
    for r in range(3):
        k = ks[freq[r]]
        re_ = e.matvec_rows(x[r], k, rows)
        rm = m.matvec_rows(x[r], k, rows, -0.5)
        assert np.linalg.norm(ye[r][rows] - re_) <= 1e-5 * np.linalg.norm(re_), r
        assert np.linalg.norm(ym[r][rows] - rm) <= 1e-5 * np.linalg.norm(rm), r
        rc = re_ + 1j / k * rm
        assert np.linalg.norm(yc[r][rows] - rc) <= 1e-5 * np.linalg.norm(rc), r
    p.close()


def test_needs_the_mesh(tmp_path):
    w = I.sphere_tiny()
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k)
    path = str(tmp_path / "plan.bin")
    p.save(path)
    q = binding.Plan.load(path)
    with pytest.raises(binding.AimError) as err:
        q.mfie_values()
    assert err.value.status == 8
    q.close()
    p.close()
