"""The paper's printed parameters (tests/golden/paper_parameters.json: the
captions of Figs. 1 and 2) converted to lattice units with the viscosity
relation of Eq. s2-ident3, nu = (tau - 1/2) dx^2 / (3 dt), and checked against
the lattice values the validation experiments run with."""
import json
import math
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_parameters.json")


def _lattice_units():
    p = json.load(open(GOLDEN))
    f1, f2 = p["fig1"], p["fig2"]
    dx, dt, rho0 = f1["dx_m"], f1["dt_s"], f1["rho0_kg_per_m3"]
    nu_lat = f1["nu_m2_per_s"] * dt / dx**2
    return {
        "tau": 3.0 * nu_lat + 0.5,
        "U": f1["U_m_per_s"] * dt / dx,
        "box": f1["box_m"] / dx,
        "R": f2["R_m"] / dx,
        "M": f2["M_kg"] / (rho0 * dx**3),
        "n": f2["n_particles"],
        "nu": nu_lat,
    }


def test_conversion_to_lattice_units():
    lu = _lattice_units()
    assert abs(lu["tau"] - 0.5534) < 1e-12
    assert abs(lu["U"] - 1e-4) < 1e-16
    assert abs(lu["box"] - 100.0) < 1e-9
    assert abs(lu["R"] - 1.0) < 1e-12
    assert abs(lu["M"] - 16.0) < 1e-9
    assert lu["n"] == 500


def test_validation_runs_use_the_printed_parameters():
    # tests/test_gpu_validation.py: Fig. 1 fluid and flow speed, Fig. 2 particle
    import test_gpu_validation as V

    lu = _lattice_units()
    assert abs(V.TAU1 - lu["tau"]) < 1e-12
    assert abs(V.U1 - lu["U"]) < 1e-16
    assert abs(V.R2 - lu["R"]) < 1e-12 and abs(V.M2 - lu["M"]) < 1e-9


def test_tail_amplitude_in_lattice_units():
    # B = M / [12 rho (pi nu)^(3/2)] of Fig. 2's caption, in steps^(3/2)
    from analytic import tail_amplitude

    lu = _lattice_units()
    gamma = 6.0 * math.pi * lu["nu"] * lu["R"]  # Stokes' law, rho = 1
    B = tail_amplitude(lu["M"], gamma, lu["R"], lu["nu"])
    assert abs(B - lu["M"] / (12.0 * (math.pi * lu["nu"]) ** 1.5)) < 1e-9 * B
    assert 100.0 < B < 101.0  # 100.83 steps^(3/2) for the paper's particle
