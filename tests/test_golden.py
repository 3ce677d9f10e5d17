"""Values printed in the paper (tests/golden/table1.json, each cited there)
against the constants the oracle and the input generators use."""
import json
import os

import pytest

import oracle
from paper_1711_04060_amd import inputs

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))


def test_oracle_constants_are_table1():
    assert (oracle.KB, oracle.TEMP, oracle.QE, oracle.EPS0_F_PER_CM) == (
        G["kB_J_per_K"], G["T_K"], G["e_C"], G["eps0_F_per_cm"])


def test_generator_constants_are_table1():
    t = inputs.TABLE1
    assert (t["kB"], t["T"], t["e"], t["eps0_F_per_cm"]) == (
        G["kB_J_per_K"], G["T_K"], G["e_C"], G["eps0_F_per_cm"])
    assert (t["eps_b"], t["eps_p"], t["eps_s"], t["eps_m"]) == (G["eps_b"], G["eps_p"], G["eps_s"], G["eps_m"])
    r = inputs.MEMBRANE_SPECIES["radius_A"]
    assert r == (G["radius_Na_A"], G["radius_Ca_A"], G["radius_Cl_A"], G["radius_H2O_A"])


def test_paper_grid_size_factorisation():
    """N = 6,246,961 is 161 x 161 x 241: a 40 x 40 x 60 A box (Eq. (4)) at
    h = 0.25 A, not the 0.5 A the text states (recorded as a reading)."""
    assert 161 * 161 * 241 == G["N_paper"]
    assert (40 / 0.25 + 1, 60 / 0.25 + 1) == (161, 241)


def test_thermal_voltage():
    assert inputs.thermal_voltage_mV() == pytest.approx(25.683, abs=1e-3)
