"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
identical seeded inputs.

Tolerances:
* FP64 storage: populations / fields / reactions to 1e-11 relative (the only
  differences are summation order and the 2^-50 fixed-point spreading);
* FP32 storage: max relative field error <= 1e-5 after 1000 steps for rho,
  u (normalised by max |u|) and T; particle positions <= 1e-4 lattice units;
* FP16 / BF16 deviation storage: reported per field, bounded as stated below.
"""
import math

import numpy as np
import pytest

from paper_1502_01159_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01159_amd import pibm

    pibm.lib()
    return pibm


def field_errors(a, b):
    """Per-field max relative errors: rho (max|rho| ~ 1), u (by max |u|), T."""
    rho, u, T = a
    r_rho, r_u, r_T = b
    eu = np.abs(u - r_u).max() / max(np.abs(r_u).max(), 1e-30)
    return dict(rho=np.abs(rho - r_rho).max() / np.abs(r_rho).max(), u=eu,
                T=np.abs(T - r_T).max() / max(np.abs(r_T).max(), 1e-30))


def reactions_close(a, b, rel, R=None):
    """Reactions F[3] tau[3] H sum(dT A): each group to `rel` of its largest
    magnitude over all particles (small components of a vector are only as
    accurate as the vector); torques also on the scale R |F|, since a torque
    that vanishes by symmetry is the difference of terms of that size."""
    fscale = np.abs(b[:, 0:3]).max()
    for lo, hi in ((0, 3), (3, 6), (6, 7), (7, 8)):
        scale = max(np.abs(b[:, lo:hi]).max(), 1e-300)
        if lo == 3 and R is not None:
            scale = max(scale, R * fscale)
        err = np.abs(a[:, lo:hi] - b[:, lo:hi]).max()
        assert err <= rel * scale, (lo, hi, err, scale)


def run_pair(gpu, oracle_mod, cfg, P, steps, storage, chunk=None):
    sim = gpu.Simulation(cfg, P, storage=storage)
    ref = oracle_mod.Oracle(cfg, P)
    sim.step(steps)
    ref.step(steps)
    assert sim.sync() == gpu.OK
    return sim, ref


def _box_particles(dim, n, seed):
    """A few bodies near walls and across the periodic seam (x periodic)."""
    rng = np.random.default_rng(seed)
    rows = []
    if dim == 2:
        cents = [(3.0, 20.5), (146.2, 10.0), (70.3, 30.1), (100.0, 6.5)]
        R = [5.5, 6.0, 4.5, 6.0]
    else:
        cents = [(3.0, 5.2, 4.9), (64.0, 5.7, 5.1), (35.2, 5.0, 5.3)]
        R = [4.0, 3.5, 4.2]
    for c, r in zip(cents, R):
        u = 0.01 * (rng.random(3) - 0.5)
        om = 0.002 * (rng.random(3) - 0.5)
        if dim == 2:
            u[2] = 0.0
            om[:2] = 0.0
        rows.append([c[0], c[1], c[2] if dim == 3 else 0.0, *u, *om, r, 1.5, float(rng.random()), 0.0])
    return np.array(rows)


@pytest.mark.parametrize("dim,order,lattice,tm", [(2, 2, 19, 0), (3, 2, 19, 0), (2, 4, 19, 0), (3, 4, 19, 0),
                                                  (3, 2, 15, 0), (2, 2, 19, 1), (3, 2, 19, 1), (3, 2, 15, 1)])
def test_single_step_random_state_f64(gpu, oracle_mod, dim, order, lattice, tm):
    """One step from a random non-equilibrium state on a ragged multi-tile
    box (x periodic, y and z walls): every population, and every particle's
    reactions and new state, agree with the oracle; with the multilinear
    (i_max = 2) and the cubic (i_max = 4) interpolation of Eq. (lbm6), on the
    D3Q15 flow lattice of Sec. 2.1, and with temperature on the flow lattice
    (quadratic equilibrium; tm = 1), walls at different temperatures meeting
    at edges."""
    if dim == 2:
        cfg = dict(dim=2, nx=150, ny=37, nz=1, periodic=[1, 0, 0])
    else:
        cfg = dict(dim=3, nx=70, ny=11, nz=10, periodic=[1, 0, 0])
    cfg.update(T_wall=[0.2, 0.7, 0.0, 1.0, 0.3, 0.6], T_init=0.4, T_ref=0.35, Ra=0.0, nu=0.05, Pr=0.7,
               Gr=300.0, Lc=8.0, gravity=2e-3, kappa_T=1.0, marker_mode=1, marker_spacing=1.0,
               E_star=50.0, poisson=0.33, mu_fric=0.3, n_sub=3, beta_p=0.05, c_r=1.0, interp_order=order,
               lattice=lattice, thermal_model=tm)
    P = _box_particles(dim, cfg["nx"], 7)
    P[0, 12] = W.THERMO
    sim = gpu.Simulation(cfg, P, storage="f64")
    ref = oracle_mod.Oracle(cfg, P)
    Q, Qg = sim.Q, sim.Qg
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4) if dim == 2 else \
        (np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8) if lattice == 15 else
         np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12))
    wg = w if tm == 1 else (np.array([1 / 3] + [1 / 6] * 4) if dim == 2 else np.array([1 / 4] + [1 / 8] * 6))
    f0 = W.perturbed_populations(11, Q, sim.N, w, 1.0, 0.05)
    g0 = W.perturbed_populations(12, Qg, sim.N, wg, 0.5, 0.2)
    sim.set_populations(f0, g0)
    ref.set_populations(f0, g0)
    fa, ga = sim.populations()
    assert np.array_equal(fa, f0) and np.array_equal(ga, g0)
    sim.step(1)
    ref.step(1)
    assert sim.sync() == gpu.OK
    f1, g1 = sim.populations()
    rf, rg = ref.populations()
    assert np.abs(f1 - rf).max() < 1e-13
    assert np.abs(g1 - rg).max() < 1e-13
    q, fth = sim.particles()
    rq = ref.particles()
    assert np.allclose(fth, ref.reactions(), rtol=1e-11, atol=1e-13)
    assert np.abs(q[:, :12] - rq[:, :12]).max() < 1e-12
    assert np.allclose(q[:, 14], rq[:, 14], rtol=1e-12, atol=1e-14)


def workload_case(name):
    """A named workload; the suffix _q15 puts it on the D3Q15 flow lattice,
    _tm1 puts the temperature on the flow lattice (quadratic equilibrium)."""
    over = {}
    if name.endswith("_tm1"):
        name, over["thermal_model"] = name[:-4], 1
    if name.endswith("_q15"):
        name, over["lattice"] = name[:-4], 15
    cfg, P = W.workload(name)
    return W.with_overrides(cfg, **over), P


@pytest.mark.parametrize("name,steps", [("c1", 2000), ("c2_small", 200), ("c3_small", 60), ("c4_small", 60),
                                        ("c3_small_q15", 60), ("c1_tm1", 300), ("c3_small_q15_tm1", 60),
                                        ("x3", 2), ("x2", 2), ("x2_noheat", 2), ("c2", 200), ("c3_mid", 200), ("c4_mid", 100)])
def test_workloads_f64(gpu, oracle_mod, name, steps):
    cfg, P = workload_case(name)
    sim, ref = run_pair(gpu, oracle_mod, cfg, P, steps, "f64")
    e = field_errors(sim.fields(), ref.fields())
    assert max(e.values()) < 1e-9, e
    q, fth = sim.particles()
    rq = ref.particles()
    assert np.abs(q[:, :3] - rq[:, :3]).max() < 1e-10
    reactions_close(fth, ref.reactions(), 1e-9, R=P[:, 9].max())
    assert np.allclose(q[:, 14], rq[:, 14], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("name,steps", [("c1", 2000), ("c2_small", 1000), ("c3_small", 1000), ("c4_small", 1000),
                                        ("c4_small_q15", 1000), ("c2", 1000), ("c3_mid", 1000), ("c4_mid", 500)])
def test_workloads_f32_1000_steps(gpu, oracle_mod, name, steps):
    """The stated FP32 bar: fields <= 1e-5 relative, positions <= 1e-4 lu,
    after 1000 steps (the annulus case over its whole 2000; the downsized
    thermosensitive case, 96^3 with 288 spheres, 500, where the oracle takes
    a quarter of a second per step)."""
    cfg, P = workload_case(name)
    sim, ref = run_pair(gpu, oracle_mod, cfg, P, steps, "f32")
    e = field_errors(sim.fields(), ref.fields())
    print(name, "f32 field errors", e)
    assert max(e.values()) <= 1e-5, e
    q, _ = sim.particles()
    rq = ref.particles()
    dx = np.abs(q[:, :3] - rq[:, :3]).max()
    print(name, "f32 max position error", dx)
    assert dx <= 1e-4


def _compare_full(gpu, ref, cfg, P, storage, steps, log):
    """A fresh full-size run of `steps` steps in `storage` against the oracle
    state `ref` (already at that step); returns per-field errors and the
    largest position error."""
    sim = gpu.Simulation(cfg, P, storage=storage)
    sim.step(steps)
    assert sim.sync() == gpu.OK
    e = field_errors(sim.fields(), log["ref_fields"])
    q, fth = sim.particles()
    dx = float(np.abs(q[:, :3] - ref.particles()[:, :3]).max())
    print("c3", storage, steps, "steps: field errors", e, "max position error", dx, flush=True)
    sim.close()
    return e, dx, fth


def test_full_size_c3_every_node(gpu, oracle_mod):
    """The benchmark's default workload itself (256 x 256 x 512, 2000 spheres,
    the two-stream step) against one oracle run on every node and particle:
    FP64 storage after 3 steps to the FP64 bar; FP32, FP16 and BF16 deviation
    storage after 4 steps (the variants the benchmark times); FP32 again
    after 50 steps.  FP32: fields <= 1e-5, positions <= 1e-4 lu.  FP16: rho,
    u and T <= 1e-3 of the FP64 result.  BF16 is reported (its 8-bit
    significand misses the 1e-3 bar at longer horizons: see the small-box
    test below) and bounded by 1e-2."""
    cfg, P = W.workload("c3")
    ref = oracle_mod.Oracle(cfg, P)
    log = {}
    ref.step(3)
    log["ref_fields"] = ref.fields()
    e, dx, fth = _compare_full(gpu, ref, cfg, P, "f64", 3, log)
    assert max(e.values()) <= 1e-9 and dx <= 1e-10, e
    reactions_close(fth, ref.reactions(), 1e-9, R=P[:, 9].max())
    ref.step(1)
    log["ref_fields"] = ref.fields()
    results = {}
    for storage in ("f32", "f16", "bf16"):
        results[storage] = _compare_full(gpu, ref, cfg, P, storage, 4, log)[:2]
    ref.step(46)
    log["ref_fields"] = ref.fields()
    results["f32_50"] = _compare_full(gpu, ref, cfg, P, "f32", 50, log)[:2]
    for key, bound, dxb in (("f32", 1e-5, 1e-4), ("f32_50", 1e-5, 1e-4), ("f16", 1e-3, 1e-3), ("bf16", 1e-2, 1e-2)):
        e, dx = results[key]
        assert max(e.values()) <= bound and dx <= dxb, (key, e, dx)


def test_full_size_c4_every_node(gpu, oracle_mod):
    """The largest workload (384^3, 20,000 thermosensitive spheres, FP32
    storage, the two-stream step) against the oracle on every node and every
    particle after 3 steps: fields <= 1e-5, positions <= 1e-4 lu, particle
    temperatures to 1e-5 of their range."""
    cfg, P = W.workload("c4")
    ref = oracle_mod.Oracle(cfg, P)
    ref.step(3)
    rf = ref.fields()
    sim = gpu.Simulation(cfg, P, storage="f32")
    sim.step(3)
    assert sim.sync() == gpu.OK
    e = field_errors(sim.fields(), rf)
    q, _ = sim.particles()
    rq = ref.particles()
    dx = float(np.abs(q[:, :3] - rq[:, :3]).max())
    dT = float(np.abs(q[:, 14] - rq[:, 14]).max())
    print("c4 f32 3 steps: field errors", e, "max position error", dx, "max particle T error", dT, flush=True)
    assert max(e.values()) <= 1e-5, e
    assert dx <= 1e-4 and dT <= 1e-5
    sim.close()


def test_packed_bed_contacts_f64(gpu, oracle_mod):
    """The DEM's contact path under load: 107 spheres settling onto each
    other and the floor (over 200 oblique pair contacts and 25 floor
    contacts at once, counted from the oracle's brute-force contact lists,
    with Coulomb-capped tangential springs), FP64 storage, 500 coupled steps
    against the oracle: fields, positions, velocities, spins, reactions."""
    cfg, P = W.workload("packed_bed")
    sim = gpu.Simulation(cfg, P, storage="f64")
    ref = oracle_mod.Oracle(cfg, P)
    for chunk in range(2):
        sim.step(250)
        ref.step(250)
        assert sim.sync() == gpu.OK
        n_pairs = sum(len(ref.contacts(i)) for i in range(len(P))) // 2
        q, fth = sim.particles()
        rq = ref.particles()
        dq = float(np.abs(q[:, :9] - rq[:, :9]).max())
        print(f"packed bed {250 * (chunk + 1)} steps: {n_pairs} pair contacts, max state error {dq:.3e}", flush=True)
        assert n_pairs >= 100
        assert dq <= 1e-9
        reactions_close(fth, ref.reactions(), 1e-9, R=P[:, 9].max())
    e = field_errors(sim.fields(), ref.fields())
    assert max(e.values()) <= 1e-9, e
    sim.close()


@pytest.mark.parametrize("storage,bound", [("f16", 1e-3), ("bf16", 1e-2)])
def test_16bit_deviation_storage_error(gpu, oracle_mod, storage, bound):
    """FP16 / BF16 deviation storage collided in FP32: per-field error against
    the FP64 oracle after 300 steps of the 3D sedimentation case.  FP16 meets
    the 1e-3 bar on rho, u and T.  BF16's 8-bit significand does not: its u
    and T errors are 3-5e-3 here, so its bound is 1e-2 and the miss is stated
    wherever BF16 is reported."""
    cfg, P = W.workload("c3_small")
    sim, ref = run_pair(gpu, oracle_mod, cfg, P, 300, storage)
    e = field_errors(sim.fields(), ref.fields())
    q, _ = sim.particles()
    dx = np.abs(q[:, :3] - ref.particles()[:, :3]).max()
    print(storage, "field errors", e, "max position error", dx)
    assert e["rho"] <= bound and e["u"] <= bound and e["T"] <= bound, e


def test_bitwise_reproducible(gpu):
    """Two runs give identical bits: the spreading accumulates in integer
    fixed point and every reduction has a fixed order."""
    cfg, P = W.workload("c3_small")
    a = gpu.Simulation(cfg, P, storage="f32")
    b = gpu.Simulation(cfg, P, storage="f32")
    a.step(40)
    b.step(40)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    qa, ra = a.particles()
    qb, rb = b.particles()
    assert np.array_equal(qa, qb) and np.array_equal(ra, rb)


def test_checkpoint_roundtrip(gpu):
    """2N steps == N steps + save + (more steps) + load + N steps, bitwise."""
    cfg, P = W.workload("c2_small")
    s = gpu.Simulation(cfg, P, storage="f32")
    s.step(25)
    blob = s.save()
    s.step(25)
    f1, g1 = s.populations()
    q1, _ = s.particles()
    s.step(7)
    s.load(blob)
    assert s.step_count == 25
    s.step(25)
    f2, g2 = s.populations()
    q2, _ = s.particles()
    assert np.array_equal(f1, f2) and np.array_equal(g1, g2) and np.array_equal(q1, q2)


def test_checkpoint_restores_16bit_storage_offset(gpu):
    """16-bit storage keeps g's deviation from an offset set by the case's
    initial temperatures.  A checkpoint carries it: a context set up with
    other particle temperatures (hence another offset) that loads the blob
    holds the same populations and continues the run bit for bit."""
    cfg, P = W.workload("c2_small")
    a = gpu.Simulation(cfg, P, storage="f16")
    a.step(20)
    blob = a.save()
    P2 = np.array(P, dtype=float)
    P2[:, 11] = 3.0                                  # particle temperatures: another offset
    b = gpu.Simulation(cfg, P2, storage="f16")
    b.load(blob)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    a.step(10)
    b.step(10)
    for x, y in zip(a.populations() + a.particles(), b.populations() + b.particles()):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_watchdog_reports_runaway_velocity(gpu):
    """A node driven past |u| = 0.4 (finite values, set from the host) trips
    the device watchdog: PIBM_EUNSTABLE, later steps are refused and the
    device stops advancing the state."""
    cfg, P = W.workload("c2_small")
    s = gpu.Simulation(cfg, P, storage="f32")
    s.step(2)
    f, g = s.populations()
    f[1, 1234] += 0.8                   # rho = 1.8, u_x = 0.44 at one node far from the disks
    s.set_populations(f, g)
    s.step(3)
    assert s.sync() == gpu.EUNSTABLE
    with pytest.raises(gpu.PibmError):
        s.step(1)


@pytest.mark.parametrize("streams", [1, 2])
def test_nan_in_particle_stencil_reports_unstable(gpu, streams):
    """Regression test of the recorded fault (non-finite particle centres gave
    out-of-range indices).  NaN populations on a row through particle 0's
    equator, inside the stencils of its Lagrangian points: the exchange gives
    NaN reactions, the lattice kernel flags its NaN node, and the DEM either
    stops at that flag (one stream) or, running beside the lattice kernel
    (two streams), flags the NaN centre itself.  Every later kernel returns at
    entry, pibm_sync reports PIBM_EUNSTABLE and the next pibm_step is refused;
    the particle state is still readable and its reactions show that the NaN
    went through the exchange."""
    cfg, P = W.workload("c3_small")
    s = gpu.Simulation(dict(cfg, streams=streams), P, storage="f32")
    s.step(3)
    assert s.sync() == gpu.OK
    f, g = s.populations()
    nx, ny = cfg["nx"], cfg["ny"]
    x0, y0, z0, R = P[0, 0], P[0, 1], P[0, 2], P[0, 9]
    j, k = int(math.floor(y0)), int(math.floor(z0))
    for i in range(int(math.floor(x0 - R)) - 1, int(math.floor(x0 + R)) + 3):
        f[3, (k * ny + j) * nx + i] = np.nan
    print(f"NaN row through particle 0 (streams {streams})", flush=True)
    s.set_populations(f, g)
    s.step(2)
    assert s.sync() == gpu.EUNSTABLE
    with pytest.raises(gpu.PibmError):
        s.step(1)
    q, fth = s.particles(check=False)
    assert not np.all(np.isfinite(fth[0]))          # the NaN went through the exchange
    assert np.all(np.isfinite(fth[1:]))             # the other particles' stencils are clean
    s.close()


@pytest.mark.parametrize("case,storage", [("c3_small", "f32"), ("c2_small", "f16"), ("c4_small", "f32")])
def test_two_streams_match_one_stream(gpu, case, storage):
    """Binning beside the exchange and the DEM beside the lattice kernel (a
    second stream) give bit-identical populations, particles and reactions to
    the one-stream order."""
    cfg, P = W.workload(case)
    out = []
    for streams in (1, 2):
        s = gpu.Simulation(dict(cfg, streams=streams), P, storage=storage)
        s.step(30)
        f, g = s.populations()
        q, r = s.particles()
        out.append((f, g, q, r))
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_neighbour_capacity_reports_enomem(gpu):
    """More neighbour candidates than a particle's list holds (32): the
    device's own bounds check stops the list at capacity and reports
    PIBM_ENOMEM; later steps are refused.  A 5^3 block of point particles at
    pitch 0.6 with skin 1 gives the central one 80 candidates."""
    cfg = dict(dim=3, nx=12, ny=12, nz=12, periodic=[1, 1, 1], T_wall=[0.0] * 6, T_init=0.0, T_ref=0.0,
               Ra=0.0, nu=0.1, Pr=0.7, Gr=0.0, Lc=8.0, gravity=0.0, kappa_T=1.0, marker_mode=2,
               marker_spacing=1.0, E_star=10.0, poisson=0.33, mu_fric=0.3, n_sub=1, beta_p=0.0, c_r=1.0,
               skin=1.0)
    P = np.array([[4.0 + 0.6 * i, 4.0 + 0.6 * j, 4.0 + 0.6 * k, 0, 0, 0, 0, 0, 0, 0.25, 1.0, 0.0, W.FIXED]
                  for i in range(5) for j in range(5) for k in range(5)])
    s = gpu.Simulation(cfg, P, storage="f32")
    s.step(1)
    assert s.sync() == gpu.ENOMEM
    with pytest.raises(gpu.PibmError):
        s.step(1)
    s.close()


def test_profile_phases(gpu):
    """Phase profiling times only the phases in the mask; the full mask times
    all four; bits beyond the phases are refused."""
    cfg, P = W.workload("c2_small")
    s = gpu.Simulation(cfg, P, storage="f32")
    s.profile(True, phases=["lattice"])
    s.step(3)
    r = s.profile_read()
    assert r["lattice"][1] == 3 and r["lattice"][0] > 0
    assert r["markers"][1] == r["bin"][1] == r["dem"][1] == 0
    s.profile(True)
    s.step(2)
    r = s.profile_read()
    assert all(r[p][1] == 2 for p in gpu.PHASES)
    s.profile(False)
    s.step(1)
    assert all(v[1] == 0 for v in s.profile_read().values())
    assert gpu.lib().pibm_profile_phases(s._h, 1 << len(gpu.PHASES)) == gpu.EINVAL
    s.close()


def test_rest_state_exact_in_f32(gpu):
    """P1 on the GPU: deviation storage keeps the rest state exactly."""
    cfg = dict(dim=3, nx=70, ny=9, nz=6, periodic=[0, 1, 0], T_wall=[0.5] * 6, T_init=0.5, T_ref=0.5,
               Ra=0.0, nu=0.05, Pr=0.7, Gr=100.0, Lc=8.0)
    s = gpu.Simulation(cfg, None, storage="f32")
    s.step(50)
    f, g = s.populations()
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=np.float32).astype(np.float64)
    assert np.array_equal(f, np.repeat(np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None], s.N, 1))
    assert np.all(g == np.repeat((np.array([1 / 4] + [1 / 8] * 6) * 0.5)[:, None], s.N, 1))
    del w


# --------------------------------------------------------------------------- #
# Full sizes, in the launch configuration the benchmark times                 #
# --------------------------------------------------------------------------- #

def _crop(cfg, P, centre, half):
    """Periodic crop of side 2*half around `centre` holding the particles that
    lie entirely inside it (so that none meets a periodic image of another:
    such spurious contacts would travel inward through the DEM sub-steps)."""
    lo = np.floor(np.array(centre) - half).astype(int)
    n = 2 * half
    c2 = dict(cfg, nx=n, ny=n, nz=n, periodic=[1, 1, 1])
    keep = []
    for r in P:
        x = r[:3] - lo
        if np.all(x >= r[9] + 1) and np.all(x <= n - r[9] - 1):
            rr = r.copy()
            rr[:3] = x
            keep.append(rr)
    return c2, np.array(keep), lo


@pytest.mark.parametrize("name", ["c3", "c4"])
def test_full_size_light_cone_samples(gpu, oracle_mod, name):
    """At the full benchmark size (FP32 storage), two coupled steps from the
    uniform rest state.  Within one step information moves at most about
    2R + 4 lattice units (streaming, interpolation, spreading, and the rigid
    particle carrying its markers' forces across its diameter), so inside a
    periodic crop around a particle near the box centre the oracle reproduces
    the full-size run away from the crop boundary: fields there and the
    centre particle's reactions are compared element by element.  Mass
    conservation over the whole lattice is checked as a property that holds
    at any size."""
    cfg, P = W.workload(name)
    steps = 2
    sim = gpu.Simulation(cfg, P, storage="f32")
    rho0 = sim.fields()[0].sum(dtype=np.float64)
    sim.step(steps)
    assert sim.sync() == gpu.OK
    rho, u, T = sim.fields()
    assert abs(rho.sum(dtype=np.float64) - rho0) / rho0 < 1e-6
    q, fth = sim.particles()
    mid = np.array([cfg["nx"] / 2, cfg["ny"] / 2, np.median(P[:, 2])])
    k = int(np.argmin(np.abs(P[:, :3] - mid).sum(1)))
    Rm = int(math.ceil(P[:, 9].max()))
    m = (steps + 1) * (2 * Rm + 4) + 2            # influence radius of steps + the fields pass
    half = m + 12
    c2, P2, lo = _crop(cfg, P, P[k, :3], half)
    ref = oracle_mod.Oracle(c2, P2)
    ref.step(steps)
    rr, ru, rT = ref.fields()
    sl = (slice(m, 2 * half - m),) * 3
    g = tuple(slice(lo[2 - a] + m, lo[2 - a] + 2 * half - m) for a in range(3))
    assert rho[g].shape == rr[sl].shape and rr[sl].size > 0
    e = field_errors((rho[g], u[g], T[g]), (rr[sl], ru[sl], rT[sl]))
    print(name, "crop field errors", e, "particles in crop", len(P2))
    assert max(e.values()) < 1e-5, e
    # reactions and new position of the particle at the crop centre
    i2 = int(np.argmin(np.linalg.norm(P2[:, :3] - (P[k, :3] - lo), axis=1)))
    assert np.allclose(fth[k], ref.reactions()[i2], rtol=2e-5, atol=2e-6)
    assert np.abs(q[k, :3] - (ref.particles()[i2, :3] + lo)).max() < 1e-6
