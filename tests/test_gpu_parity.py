"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances: complex128 path <= 1e-10 relative L2, complex64 path <= 1e-5
relative L2 (both against the float64 oracle); per-stage complex128 results
are compared at rounding level; integer/index work bit-exact."""
import math

import numpy as np
import pytest

from paper_2009_02281_amd import inputs as I
from oracle import aimx, excitation

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU machines skip the module
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402

FP64_TOL = 1e-10
FP32_TOL = 1e-5


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


_CACHE = {}


def _setup(name):
    if name not in _CACHE:
        w = {"sphere": I.sphere_small, "boxes": I.small_box_array}[name]()
        o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
        o.C
        p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                         max_rhs=8)
        _CACHE[name] = (w, o, p)
    return _CACHE[name]


CASES = ["sphere", "boxes"]


@pytest.mark.parametrize("case", CASES)
def test_stage_project(case):
    w, o, p = _setup(case)
    print(f"[gpu] project {case} N={o.N}", flush=True)
    x = I.complex_gaussian(o.N, 101, nrhs=3)
    q = host(p.apply_stage("project", dev(x)))
    ref = o.project(x)
    assert rel(q, ref) <= 1e-14
    qf = host(p.apply_stage("project", dev(x, torch.complex64), prec="c64"))
    assert rel(qf, ref) <= 1e-6


@pytest.mark.parametrize("case", CASES)
def test_stage_convolve(case):
    w, o, p = _setup(case)
    print(f"[gpu] convolve {case} dims={o.dims}", flush=True)
    Nx, Ny, Nz = o.dims
    g = I.complex_gaussian(Nx * Ny * Nz, 102, nrhs=2).reshape(2, Nz, Ny, Nx)
    phi = host(p.apply_stage("convolve", dev(g)))
    ref = aimx.grid_convolve(g, o.spectrum(w.k[0]), o.dims)
    assert rel(phi, ref) <= 1e-12
    phif = host(p.apply_stage("convolve", dev(g, torch.complex64), prec="c64"))
    assert rel(phif, ref) <= FP32_TOL


@pytest.mark.parametrize("case", CASES)
def test_stage_interpolate_and_near(case):
    w, o, p = _setup(case)
    print(f"[gpu] interpolate/near {case}", flush=True)
    Nx, Ny, Nz = o.dims
    g = I.complex_gaussian(Nx * Ny * Nz, 103, nrhs=2).reshape(2, Nz, Ny, Nx)
    y = host(p.apply_stage("interpolate", dev(g)))
    assert rel(y, o.interpolate(g)) <= 1e-14
    x = I.complex_gaussian(o.N, 104, nrhs=2)
    yn = host(p.apply_stage("near", dev(x)))
    assert rel(yn, (o.C @ x.T).T) <= 1e-14


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("nrhs", [1, 5])
def test_matvec_fp64_and_fp32(case, nrhs):
    w, o, p = _setup(case)
    print(f"[gpu] matvec {case} nrhs={nrhs}", flush=True)
    x = I.complex_gaussian(o.N, 1001, nrhs=nrhs)
    ref = o.matvec(x, w.k[0])
    y64 = host(p.matvec(dev(x)))
    assert rel(y64, ref) <= FP64_TOL
    y32 = host(p.matvec(dev(x, torch.complex64), prec="c64"))
    e32 = rel(y32, ref)
    print(f"    fp64 err {rel(y64, ref):.2e}  fp32 err {e32:.2e}", flush=True)
    assert e32 <= FP32_TOL


def test_matvec_frequency_batch():
    """Several wavenumbers in one plan; each right-hand side selects its own
    kernel spectrum (the batched sweep)."""
    w = I.sweep_small(nfreq=6, rhs_per_freq=2)
    print("[gpu] frequency batch", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=12)
    freq = np.repeat(np.arange(6), 2)[::-1].copy()
    x = I.complex_gaussian(o.N, 3001, nrhs=12)
    y64 = host(p.matvec(dev(x), freq_idx=freq))
    y32 = host(p.matvec(dev(x, torch.complex64), freq_idx=freq, prec="c64"))
    for r in range(12):
        ref = o.matvec(x[r], w.k[freq[r]])
        assert rel(y64[r], ref) <= FP64_TOL
        assert rel(y32[r], ref) <= FP32_TOL
    p.close()


def test_many_right_hand_sides_at_many_wavenumbers():
    """61 vectors at 8 wavenumbers (workgroups serve several vectors each,
    the last one fewer), every vector against the oracle, in the four stage
    modes (both interpolations, the projection on its own or fused into the
    x forward pass)."""
    w = I.sweep_small(nfreq=8, rhs_per_freq=8)
    print("[gpu] 64 right-hand sides", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=64)
    nv = 61                     # not a multiple of the vectors per workgroup
    freq = np.arange(nv) % 8
    x = I.complex_gaussian(o.N, 3101, nrhs=nv)
    refs = [o.matvec(x[r], w.k[freq[r]]) for r in range(nv)]
    for mode in (0, 1, 2, 3):
        for prec, dt, tol in (("c128", torch.complex128, FP64_TOL),
                              ("c64", torch.complex64, FP32_TOL)):
            p.set_schedule([0] * 6 + [mode], prec=prec)
            y = host(p.matvec(dev(x, dt), freq_idx=freq, prec=prec))
            for r in range(nv):
                assert rel(y[r], refs[r]) <= tol, (mode, prec, r)
    p.close()


def test_projection_is_deterministic():
    w, o, p = _setup("boxes")
    x = dev(I.complex_gaussian(o.N, 105, nrhs=4))
    a = p.apply_stage("project", x)
    b = p.apply_stage("project", x)
    assert torch.equal(a, b)
    ya = p.matvec(x)
    yb = p.matvec(x)
    assert torch.equal(ya, yb)
    p.set_schedule([0] * 6 + [2])        # projection inside the x forward pass
    yf = p.matvec(x)
    assert torch.equal(yf, p.matvec(x))
    assert rel(host(yf), host(ya)) <= 1e-14
    p.set_schedule([0] * 7)


def test_operator_symmetry_on_gpu():
    w, o, p = _setup("sphere")
    x = I.complex_gaussian(o.N, 11)
    y = I.complex_gaussian(o.N, 12)
    Ay = host(p.matvec(dev(y)))
    Ax = host(p.matvec(dev(x)))
    assert abs(x @ Ay - y @ Ax) <= 1e-12 * abs(x @ Ay)
    Ay32 = host(p.matvec(dev(y, torch.complex64), prec="c64"))
    Ax32 = host(p.matvec(dev(x, torch.complex64), prec="c64"))
    assert abs(x @ Ay32 - y @ Ax32) <= 1e-6 * abs(x @ Ay32)


def test_excitation_matches_oracle():
    w, o, p = _setup("sphere")
    b = host(p.excitation("plane_wave", [0.0, 0.0, 1.0]))[0]
    assert rel(b, excitation.plane_wave(o.V, o.T, w.k[0])) <= 1e-14
    c = o.cent[17]
    g = host(p.excitation("gaussian_patch", [c[0], c[1], c[2], 0.2]))[0]
    assert rel(g, excitation.gaussian_patch(o.V, o.T, c, 0.2)) <= 1e-14


def test_invalid_calls_raise():
    w, o, p = _setup("sphere")
    x = dev(I.complex_gaussian(o.N, 1, nrhs=9))
    with pytest.raises(binding.AimError) as e:
        p.matvec(x)                     # nrhs above max_rhs
    assert e.value.status == 1
    with pytest.raises(binding.AimError):
        p.matvec(x[:2], freq_idx=[0, 3])   # frequency index out of range


def test_full_size_box_array_shared_blocks():
    """The full-size box array with 7 right-hand sides: the projection and
    interpolation workgroups each serve several right-hand sides.  Sampled
    rows of every vector against the oracle, both precisions and the four
    stage modes."""
    w = I.box_array_large()
    print("[gpu] full-size box array, 7 right-hand sides", flush=True)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=8)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    x = I.complex_gaussian(o.N, 2101, nrhs=7)   # 4 + 3 vectors per workgroup
    rows = np.sort(np.random.default_rng(2102).choice(o.N, 16, replace=False))
    refs = [o.matvec_rows(x[r], w.k[0], rows) for r in range(7)]
    for mode in (0, 1, 2, 3):
        for prec, dt, tol in (("c128", torch.complex128, FP64_TOL),
                              ("c64", torch.complex64, FP32_TOL)):
            p.set_schedule([0] * 6 + [mode], prec=prec)
            y = host(p.matvec(dev(x, dt), prec=prec))
            for r in range(7):
                assert rel(y[r][rows], refs[r]) <= tol, (mode, prec, r)
    p.close()


def test_full_size_box_array_sampled():
    """The 4x4 box array at full size (57,600 triangles, 128x128x64 grid,
    3rd-order stencils) in the configuration the benchmark times: all rows of
    the far part and sampled rows of the full product against the oracle."""
    w = I.box_array_large()
    print(f"[gpu] full-size box array N={w.n}", flush=True)
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=1)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    x = I.complex_gaussian(o.N, 2001)
    rows = np.sort(np.random.default_rng(2002).choice(o.N, 48, replace=False))
    ref = o.matvec_rows(x, w.k[0], rows)
    y64 = host(p.matvec(dev(x)))
    y32 = host(p.matvec(dev(x, torch.complex64), prec="c64"))
    assert rel(y64[rows], ref) <= FP64_TOL
    assert rel(y32[rows], ref) <= FP32_TOL
    far = o.far(x, w.k[0])
    q = p.apply_stage("project", dev(x))
    yfar = host(p.apply_stage("interpolate", p.apply_stage("convolve", q)))
    assert rel(yfar[0], far) <= FP64_TOL
    print(f"    fp64 err {rel(y64[rows], ref):.2e} fp32 err {rel(y32[rows], ref):.2e}", flush=True)
    p.close()


@pytest.mark.parametrize("case", CASES)
def test_implicit_interpolation_matches_oracle(case):
    """Interpolation with the weights of P^T recomputed from the quadrature
    points (schedule entry 6 = 1): stage and whole-matvec parity, both
    precisions."""
    w, o, p = _setup(case)
    Nx, Ny, Nz = o.dims
    g = I.complex_gaussian(Nx * Ny * Nz, 113, nrhs=2).reshape(2, Nz, Ny, Nx)
    x = I.complex_gaussian(o.N, 114, nrhs=3)
    ref_y = o.matvec(x, w.k[0])
    for prec, dt, tol in (("c128", torch.complex128, FP64_TOL), ("c64", torch.complex64, FP32_TOL)):
        p.set_schedule([0] * 6 + [1], prec=prec)
        y = host(p.apply_stage("interpolate", dev(g, dt), prec=prec))
        assert rel(y, o.interpolate(g)) <= (1e-14 if prec == "c128" else 1e-6)
        assert rel(host(p.matvec(dev(x, dt), prec=prec)), ref_y) <= tol
        p.set_schedule([0] * 7, prec=prec)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_every_fft_launch_shape_matches_oracle(prec):
    """Each launch shape of each FFT pass, in every workspace layout, gives
    the oracle's result."""
    w, o, p = _setup("boxes")
    dt = torch.complex128 if prec == "c128" else torch.complex64
    tol = FP64_TOL if prec == "c128" else FP32_TOL
    x = I.complex_gaussian(o.N, 77, nrhs=3)
    ref = o.matvec(x, w.k[0])
    xd = dev(x, dt)
    tried = 0
    for layout in range(binding.FFT_LAYOUTS):
        for k in range(5):
            for v in range(binding.FFT_SHAPES):
                sched = [0] * 5 + [layout]
                sched[k] = v
                try:
                    p.set_schedule(sched, prec=prec)
                except binding.AimError:
                    continue
                tried += 1
                assert rel(host(p.matvec(xd, prec=prec)), ref) <= tol, (k, v, layout)
                if k == 0:           # the same x forward shape with the projection fused
                    p.set_schedule(sched + [2], prec=prec)
                    assert rel(host(p.matvec(xd, prec=prec)), ref) <= tol, (v, layout, "fused")
    assert tried >= 16 * binding.FFT_LAYOUTS
    with pytest.raises(binding.AimError):
        p.set_schedule([0] * 5 + [binding.FFT_LAYOUTS], prec=prec)
    res = p.autotune(prec=prec, nrhs=3, reps=3)
    assert len(res["schedule"]) == binding.SCHEDULE_LEN and all(t > 0 for t in res["pass_ms"])
    assert rel(host(p.matvec(xd, prec=prec)), ref) <= tol
    p.set_schedule([0] * 7, prec=prec)


def test_captured_graph_replays_match_eager():
    """A captured matvec graph, replayed several times with eager work and
    synchronisations in between, gives the eager result every time."""
    w, o, p = _setup("sphere")
    x = dev(I.complex_gaussian(o.N, 88, nrhs=4))
    y_eager = p.matvec(x)
    y = torch.empty_like(x)
    g = p.capture_matvec(x, y)
    for rep in range(4):
        y.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager), rep
        p.matvec(x[:2])           # unrelated eager work between replays
        torch.cuda.synchronize()
    x2 = dev(I.complex_gaussian(o.N, 89, nrhs=4))
    x.copy_(x2)                    # new input in the captured buffer
    g.launch()
    torch.cuda.synchronize()
    assert rel(host(y), o.matvec(host(x2), w.k[0])) <= FP64_TOL
    g.close()


def test_plan_checkpoint_gives_identical_matvecs(tmp_path):
    """A plan rebuilt from aim_plan_save output (tables and tuned schedule)
    gives bit-identical matvecs to the plan it was saved from."""
    w, o, p = _setup("boxes")
    p.autotune(prec="c64", nrhs=2, reps=2)
    path = tmp_path / "boxes.aim"
    p.save(path)
    q = binding.Plan.load(path)
    assert q.n == p.n and q.dims == p.dims and q.max_rhs == p.max_rhs
    x = I.complex_gaussian(o.N, 4001, nrhs=2)
    for prec, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        xd = dev(x, dt)
        assert torch.equal(p.matvec(xd, prec=prec), q.matvec(xd, prec=prec)), prec
    assert rel(host(q.matvec(dev(x))), o.matvec(x, w.k[0])) <= FP64_TOL
    q.close()
    p.set_schedule([0] * 7, prec="c64")


def test_profile_matvec_times_every_kernel_and_leaves_the_product():
    """aim_profile_matvec: seven positive kernel durations, and y_dev holds
    the same product as an ordinary matvec (the repeated timing launches
    overwrite the workspace first)."""
    w, o, p = _setup("boxes")
    x = dev(I.complex_gaussian(o.N, 171, nrhs=2))
    y = torch.empty_like(x)
    ms = p.profile_matvec(x, reps=4, out=y)
    assert list(ms) == binding.KERNELS and all(v > 0 for v in ms.values())
    assert torch.equal(y, p.matvec(x))


def test_full_size_autotuned_schedules_match_oracle():
    """The full-size workloads in the launch configuration the benchmark
    times: schedules picked by the autotuner (box array and the radius-6
    sphere, each in both precisions), 64 sampled rows against the oracle --
    for the sphere this covers the complex128 schedules at L = 512 and the
    256^3 projection and interpolation that the refinement's residual uses."""
    cases = [("box array", I.box_array_large, ("c128", "c64"), 2301),
             ("sphere", I.sphere_large, ("c128", "c64"), 2401)]
    for name, make, precs, seed in cases:
        w = make()
        print(f"[gpu] autotuned full size: {name} N={w.n}", flush=True)
        o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
        x = I.complex_gaussian(o.N, seed)
        rows = np.sort(np.random.default_rng(seed + 1).choice(o.N, 64, replace=False))
        ref = o.matvec_rows(x, w.k[0], rows)
        p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                         precisions=precs, max_rhs=1)
        for prec in precs:
            dt = torch.complex128 if prec == "c128" else torch.complex64
            tol = FP64_TOL if prec == "c128" else FP32_TOL
            sched = p.autotune(prec=prec, nrhs=1, reps=3)["schedule"]
            err = rel(host(p.matvec(dev(x, dt), prec=prec)).reshape(-1)[rows], ref)
            print(f"    {prec} schedule {sched}: {err:.2e}", flush=True)
            assert err <= tol, (name, prec, sched)
        p.close()


def test_sweep_batch_of_512_in_benchmark_configuration():
    """The sweep as the benchmark runs it: 512 vectors, vector r at wavenumber
    r mod 64, in one launch per kernel with autotuned schedules; 16 sampled
    vectors against the oracle at their own wavenumber, both precisions."""
    w = I.sweep_small()
    nf = len(w.k)
    print(f"[gpu] sweep batch: N={w.n}, {nf} wavenumbers, 512 vectors", flush=True)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    freq = np.arange(512) % nf
    x = I.complex_gaussian(o.N, 2501, nrhs=512)
    pick = np.sort(np.random.default_rng(2502).choice(512, 16, replace=False))
    refs = {r: o.matvec(x[r], w.k[freq[r]]) for r in pick}
    p = binding.Plan(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold, w.k,
                     max_rhs=512)
    for prec, dt, tol in (("c128", torch.complex128, FP64_TOL), ("c64", torch.complex64, FP32_TOL)):
        sched = p.autotune(prec=prec, nrhs=512, reps=2)["schedule"]
        y = host(p.matvec(dev(x, dt), freq_idx=freq, prec=prec))
        worst = max(rel(y[r], refs[r]) for r in pick)
        print(f"    {prec} schedule {sched}: worst {worst:.2e}", flush=True)
        assert worst <= tol, (prec, sched)
    p.close()
