"""Conventional AIM on the GPU (Sec. II-B): the per-wavenumber complex near
correction C(k) = A_NR(k) - A_P(k) filled on the device, and the matvec
W H(k) P x + C(k) x, against the oracle (oracle/conventional.py).
Tolerances as for AIMx: complex128 <= 1e-10 relative L2 (the correction
itself at 1e-13 of its largest entry), complex64 <= 1e-5."""
import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx
from oracle.conventional import ConventionalAim

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU machines skip the module
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("make", [I.sphere_small, I.small_box_array])
def test_conventional_correction_and_matvec_match_oracle(make):
    w = make()
    ks = [float(w.k[0]), 0.6 * float(w.k[0])]
    print(f"[gpu] conventional AIM {make.__name__} k={ks}", flush=True)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, ks,
                     max_rhs=3)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    conv = ConventionalAim(o)
    x = I.complex_gaussian(o.N, 4242, nrhs=3)
    xd = torch.from_numpy(x).cuda()
    with pytest.raises(binding.AimError):
        p.matvec_conventional(xd)             # nothing filled yet
    for f, k in enumerate(ks):
        p.conventional_fill(f)
        Ck = conv.correction(k).tocsr()
        Ck.sort_indices()
        got = p.conventional_values()
        assert got.shape == Ck.data.shape
        assert np.max(np.abs(got - Ck.data)) <= 1e-13 * np.max(np.abs(Ck.data))
        ref = conv.matvec(x, k)
        y = p.matvec_conventional(xd).cpu().numpy()
        assert rel(y, ref) <= 1e-10
        y32 = p.matvec_conventional(xd.to(torch.complex64), prec="c64").cpu().numpy()
        assert rel(y32, ref) <= 1e-5
        # the AIMx matvec of the same plan is unchanged by the fill
        ya = p.matvec(xd, freq_idx=[f] * 3).cpu().numpy()
        assert rel(ya, o.matvec(x, k)) <= 1e-10
    p.close()
