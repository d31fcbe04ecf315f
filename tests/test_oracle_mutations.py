"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of ``oracle/pibm_oracle.c`` (a sign,
a dropped factor, a transposed cross product, a wrong moment of inertia or
density ratio), compiles that copy on the CPU, and runs the pin that guards
the term against it: the pin must fail.  The unmodified oracle passes the
same pins in ``test_oracle_pins.py``.  Every fragment must occur exactly once
in the source, so a change to the oracle that moves a guarded term makes
this test fail loudly instead of silently testing nothing.
"""
import os
import types

import pytest

from tests import test_oracle_pins as pins

# (id, fragment of the oracle, planted replacement, pin, pin arguments)
MUTANTS = [
    # Eq. (demgov): reduced gravity (sign, density ratio) and rho_p(T) of Sec. 3.4
    ("gravity_sign", "gv[up] = -s->p.gravity * (1.0 - 1.0 / rho_p);", "gv[up] = s->p.gravity * (1.0 - 1.0 / rho_p);",
     pins.test_free_fall_reduced_gravity, dict(dim=3, thermo=False)),
    ("density_ratio_inverted", "gv[up] = -s->p.gravity * (1.0 - 1.0 / rho_p);",
     "gv[up] = -s->p.gravity * (1.0 - rho_p);", pins.test_free_fall_reduced_gravity, dict(dim=2, thermo=False)),
    ("beta_p_sign", "rho_p = q->rho_r * (1.0 - s->p.beta_p * (q->T - s->p.T_ref));",
     "rho_p = q->rho_r * (1.0 + s->p.beta_p * (q->T - s->p.T_ref));", pins.test_free_fall_reduced_gravity,
     dict(dim=3, thermo=True)),
    ("thermo_density_ignored", "if (q->flags & ORC_THERMO) rho_p =", "if (0) rho_p =",
     pins.test_free_fall_reduced_gravity, dict(dim=2, thermo=True)),
    # moments of inertia and contact torques (Sec. 2.3)
    ("sphere_inertia", "0.5 * m * q->R * q->R : 0.4 * m * q->R * q->R", "0.5 * m * q->R * q->R : 0.5 * m * q->R * q->R",
     pins.test_sliding_on_floor_conserves_contact_angular_momentum, dict(dim=3)),
    ("disk_inertia", "0.5 * m * q->R * q->R : 0.4 * m * q->R * q->R", "0.4 * m * q->R * q->R : 0.4 * m * q->R * q->R",
     pins.test_sliding_on_floor_conserves_contact_angular_momentum, dict(dim=2)),
    ("contact_torque_sign", "Tc[1] = rn[2]*Ft[0] - rn[0]*Ft[2];", "Tc[1] = rn[0]*Ft[2] - rn[2]*Ft[0];",
     pins.test_sliding_on_floor_conserves_contact_angular_momentum, dict(dim=3)),
    ("contact_lever_arm", "double rn[3] = {qi->R * n[0], qi->R * n[1], qi->R * n[2]};",
     "double rn[3] = {Rstar * n[0], Rstar * n[1], Rstar * n[2]};", pins.test_pair_contact_torque_lever_arms, {}),
    # Eq. (lbm13): the fluid torque, and the rigid velocity of the points
    ("fluid_torque_sign", "Ts[0] -= r[1]*FA[2] - r[2]*FA[1];", "Ts[0] += r[1]*FA[2] - r[2]*FA[1];",
     pins.test_interpolation_exact_for_linear_fields, dict(dim=3)),
    ("fluid_torque_transposed", "Ts[1] -= r[2]*FA[0] - r[0]*FA[2];", "Ts[1] -= r[0]*FA[2] - r[2]*FA[0];",
     pins.test_rotlet_torque_spinning_sphere, {}),
    ("fluid_torque_2d", "Ts[2] -= r[0]*FA[1] - r[1]*FA[0];", "Ts[2] -= r[1]*FA[0] - r[0]*FA[1];",
     pins.test_interpolation_exact_for_linear_fields, dict(dim=2)),
    ("rigid_velocity_sign", "U[0] = q->u[0] + q->om[1]*r[2] - q->om[2]*r[1];",
     "U[0] = q->u[0] - q->om[1]*r[2] + q->om[2]*r[1];", pins.test_rotlet_torque_spinning_sphere, {}),
    # the one-point step with prescribed reactions: the fluid takes -F
    ("prescribed_force_sign", "double FA[3] = {-r[0], -r[1], s->p.dim == 2 ? 0.0 : -r[2]};",
     "double FA[3] = {r[0], r[1], s->p.dim == 2 ? 0.0 : r[2]};", pins.test_prescribed_point_step_conserves_and_applies,
     dict(dim=3)),
    # one point per sub-grid particle: its cross-section per unit depth in 2D (Sec. 2.2)
    ("point_weight_2d", "q->area[0] = s->p.dim == 2 ? D : 0.25 * pi * D * D;", "q->area[0] = 0.25 * pi * D * D;",
     pins.test_point_particle_first_step_relaxation_2d, dict(d=0.25, rho_r=1.01)),
    # Eqs. (lbm7)-(lbm8): the exchange factor 2
    ("exchange_factor", "Fl[d] = 2.0 * (rl * U[d] - jl[d]);", "Fl[d] = (rl * U[d] - jl[d]);",
     pins.test_interpolation_exact_for_linear_fields, dict(dim=3)),
    # Eq. (lbm9) and the moments after Eq. (lbm3.5): half-force terms
    ("guo_prefactor", "return (1.0 - 0.5 / s->p.tau_f) * s->w[a] * acc;", "return (1.0 - 1.0 / s->p.tau_f) * s->w[a] * acc;",
     pins.test_uniform_force_adds_exact_momentum, dict(dim=3)),
    ("half_source_T", "*T = s->S[n] + 0.5 * s->QB[n];", "*T = s->S[n] + s->QB[n];",
     pins.test_heat_conserved_with_thermosensitive_particles, {}),
    ("half_force_u", "u[d] = (s->j[3*n + d] + 0.5 * F[d]) / *rho;", "u[d] = (s->j[3*n + d] + F[d]) / *rho;",
     pins.test_poiseuille_magic_tau_exact, dict(dim=2)),
    # Eq. (lbm12): the cosine kernel
    ("delta_h_width", "return 0.25 * (1.0 + cos(0.5 * pi * a));", "return 0.25 * (1.0 + cos(pi * a));",
     pins.test_delta_h_closed_forms, {}),
    # walls: anti-bounce-back Dirichlet temperature
    ("anti_bounce_back_sign", "= -s->g[n*s->Qg + s->oppg[a]] + 2.0 * s->wg[a] * s->p.T_wall[face];",
     "= s->g[n*s->Qg + s->oppg[a]] + 2.0 * s->wg[a] * s->p.T_wall[face];",
     pins.test_conduction_between_dirichlet_walls, dict(dim=2, thermal_model=0)),
    # Hertz normal force (Sec. 2.3)
    ("hertz_exponent", "double Fn = 4.0 / 3.0 * E * sqrt(Rstar) * delta * sqrt(delta);",
     "double Fn = 4.0 / 3.0 * E * sqrt(Rstar) * delta;", pins.test_hertz_head_on_impact, dict(dim=3)),
]


@pytest.fixture(scope="module")
def oracle_source(oracle_mod):
    with open(oracle_mod.SRC_PATH) as fh:
        return fh.read()


@pytest.mark.parametrize("mid,old,new,pin,kw", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(oracle_mod, oracle_source, tmp_path, mid, old, new, pin, kw):
    assert oracle_source.count(old) == 1, f"{mid}: fragment not found exactly once in the oracle"
    src = tmp_path / f"mutant_{mid}.c"
    src.write_text(oracle_source.replace(old, new))
    so = oracle_mod.compile_library(str(src), str(tmp_path / f"mutant_{mid}.so"))
    L = oracle_mod.load(so)
    mutant = types.SimpleNamespace(
        Oracle=lambda cfg, particles=None: oracle_mod.Oracle(cfg, particles, library=L),
        delta_h=lambda a: L.orc_delta_h(float(a)),
    )
    failed = False
    try:
        pin(mutant, **kw)
    except Exception:          # an assertion, or a NaN / complex value the pin could not compare
        failed = True
    assert failed, f"pin {pin.__name__}{kw} passes with the planted mistake {mid!r}"
    assert os.path.exists(so)
