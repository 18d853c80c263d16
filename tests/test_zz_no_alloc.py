"""The matvec entry point that allocates nothing (aim_matvec_static) against
aim_matvec, through the C ABI: same results on two calls in a row (the
second with fewer vectors, so stale scratch from the first call would show),
in both precisions, on a plain and a schedule-tuned plan; sizes beyond the
fixed scratch array are rejected before any launch."""
import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU machines skip the module
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402

FP64_TOL = 1e-10
FP32_TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("case", ["sphere", "boxes"])
def test_static_matvec_matches_matvec_on_successive_calls(case):
    w = {"sphere": I.sphere_small, "boxes": I.small_box_array}[case]()
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=6)
    for prec, dt, tol in (("c128", torch.complex128, FP64_TOL),
                          ("c64", torch.complex64, FP32_TOL)):
        for tuned in (False, True):
            if tuned:
                p.autotune(prec=prec, nrhs=4, reps=2)
            for call, nrhs in enumerate((5, 2)):
                print(f"[gpu] no-alloc matvec {case} {prec} tuned={tuned} call {call} "
                      f"nrhs={nrhs}", flush=True)
                x = torch.from_numpy(I.complex_gaussian(p.n, 300 + 10 * call, nrhs=nrhs)).to(dt)
                x = x.cuda()
                ref = p.matvec(x, prec=prec).cpu().numpy()
                y = torch.full_like(x, float("nan"))
                p.matvec_static(x, prec=prec, out=y)
                got = y.cpu().numpy()
                assert np.all(np.isfinite(got))
                assert rel(got, ref) <= tol
                # same kernels, same schedule, same order of operations
                assert np.array_equal(got, ref)
    p.close()


def test_static_matvec_rejects_sizes_beyond_its_scratch():
    w = I.sphere_small()
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=200)
    # complex128 needs 16 bytes x (Ng + ~6 Ng) per vector: 200 vectors of a
    # 16^3 grid exceed 64 MiB
    x = torch.zeros(200, p.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.AimError, match="scratch"):
        p.matvec_static(x)
    # the matvec with the plan's own workspace still serves that size
    y = p.matvec(x)
    assert torch.count_nonzero(y).item() == 0
    p.close()
