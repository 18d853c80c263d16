"""The linear-term modification on the GPU (Sec. III-A, eqs. linterm and
Lmatdecomplin): the device-computed diagonal D against the oracle, the
matvec with k^2 D x added (per right-hand side wavenumber), a solve of the
modified operator checked by its true residual, and switching it off."""
import math

import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx
from oracle.lin import lin_diagonal, matvec_with_lin

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU machines skip the module
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("make", [I.sphere_small, I.small_box_array])
def test_lin_term_diagonal_matvec_and_solve(make):
    w = make()
    ks = [float(w.k[0]), 10.0]
    print(f"[gpu] linear term {make.__name__}", flush=True)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, ks,
                     max_rhs=2)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    D = lin_diagonal(o)
    Dg = p.lin_diagonal()
    assert np.max(np.abs(Dg - D)) <= 1e-12 * np.max(np.abs(D))
    x = I.complex_gaussian(o.N, 31, nrhs=2)
    ref = np.stack([matvec_with_lin(o, D, x[r], ks[r]) for r in range(2)])
    p.set_lin_term(True)
    y = p.matvec(torch.from_numpy(x).cuda(), freq_idx=[0, 1]).cpu().numpy()
    assert rel(y, ref) <= 1e-10
    y32 = p.matvec(torch.from_numpy(x).to(torch.complex64).cuda(), prec="c64",
                   freq_idx=[0, 1]).cpu().numpy()
    assert rel(y32, ref) <= 1e-5
    b = p.excitation("plane_wave", [0.0, 0.0, 1.0])
    xs, res = p.solve(b, rtol=1e-8, restart=30, max_iter=2000, pc="diag")
    bh = b.cpu().numpy()[0]
    r = np.linalg.norm(bh - matvec_with_lin(o, D, xs.cpu().numpy()[0], ks[0])) / np.linalg.norm(bh)
    assert res.converged.all() and r <= 1.05e-8
    p.set_lin_term(False)
    y = p.matvec(torch.from_numpy(x).cuda(), freq_idx=[0, 1]).cpu().numpy()
    plain = np.stack([o.matvec(x[r], ks[r]) for r in range(2)])
    assert rel(y, plain) <= 1e-10
    p.close()


def test_lin_term_unavailable_without_device_fill():
    w = I.sphere_tiny()
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     host_only=True)
    with pytest.raises(binding.AimError):
        p.set_lin_term(True)
    p.close()
