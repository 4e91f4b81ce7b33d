"""Planted mistakes in copies of the oracle source must each fail at least one pin.

The mistakes are typical slips in the Sec. II formulas (a dropped term, a wrong
sign, a wrong index, a transposed operand, a wrong weight or prefactor).  Each
mutant is compiled on the CPU into a temporary directory and the pins are run
against it; the real oracle is never modified.
"""
import os

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "rad_oracle.c")

MUTATIONS = {
    "D_sign_ny_vy": ("c0 + th2 / 2.0 - dvz - nx * vx - ny * vy;", "c0 + th2 / 2.0 - dvz - nx * vx + ny * vy;"),
    "D_drop_th2": ("c0 + th2 / 2.0 - dvz - nx * vx - ny * vy;", "c0 - dvz - nx * vx - ny * vy;"),
    "g_power": ("1.0 / (den * den)", "1.0 / den"),
    "C_sign_th2": ("-th2 / 2.0 - dvz + c0;", "th2 / 2.0 - dvz + c0;"),
    "C_sign_c0": ("-th2 / 2.0 - dvz + c0;", "-th2 / 2.0 - dvz - c0;"),
    "fx_index": ("(az + ny * ay) * (nx - vx)", "(az + nx * ay) * (nx - vx)"),
    "fx_transpose": ("(az + ny * ay) * (nx - vx)", "(az + ny * ay) * (vx - nx)"),
    "fx_wrong_bracket": ("(ny * (ny - vy) + C) * ax", "(nx * (nx - vx) + C) * ax"),
    "fy_sign": ("(az + nx * ax) * (ny - vy)", "(az - nx * ax) * (ny - vy)"),
    "fy_drop_C": ("(nx * (nx - vx) + C) * ay", "(nx * (nx - vx)) * ay"),
    "fz_sign": ("C * (nx * ax + ny * ay)", "C * (nx * ax - ny * ay)"),
    "fz_drop_term": ("(nx * (nx - vx) + ny * (ny - vy)) * az", "(nx * (nx - vx)) * az"),
    "q_sign_az": ("(nx * ax + ny * ay + az) * g", "(nx * ax + ny * ay - az) * g"),
    "q_drop_ny": ("(nx * ax + ny * ay + az) * g", "(nx * ax + az) * g"),
    "psi_sign_dz": ("* s->t[k] - s->dz[k]", "* s->t[k] + s->dz[k]"),
    "psi_index_y": ("- ny * s->y[k];", "- nx * s->y[k];"),
    "psi_th2_half": ("(c0 + th2 / 2.0) * s->t[k]", "(c0 + th2) * s->t[k]"),
    "trap_end_weight": ("if (k == 0) return 0.5 * (s->t[1] - s->t[0]);",
                        "if (k == 0) return (s->t[1] - s->t[0]);"),
    "acc_cos_for_sin": ("azi += wk * fz * sn;", "azi += wk * fz * c;"),
    "spin0_weight": ("s0 = pref * (Es / E) * S;", "s0 = pref * (E / Es) * S;"),
    "spinhalf_weight": ("(Es * Es + E * E) / (2.0 * E * E) * S", "(Es * Es + E * E) / (2.0 * Es * E) * S"),
    "j_weight": ("e_ph * e_ph / (2.0 * E * E * gamma * gamma)", "e_ph * e_ph / (2.0 * E * E * gamma)"),
    "kstar": ("k * E / Es;", "k * Es / E;"),
    "forbidden": ("if (e_ph < energy_eV) {", "if (e_ph < 2.0 * energy_eV) {"),
    "S_drop_z": ("A[2] * A[2] + A[3] * A[3] +\n                             A[4] * A[4] + A[5] * A[5];\n            out_c",
                 "A[2] * A[2] + A[3] * A[3];\n            out_c"),
    "prefactor": ("ORACLE_ALPHA / (4.0 * ORACLE_PI * ORACLE_PI)", "ORACLE_ALPHA / (4.0 * ORACLE_PI)"),
    "hbarc": ("1.973269804e-7;", "1.97327e-7;"),
}


def _run_pins():
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin()
        except Exception as e:  # a failing assertion, or a NaN-driven error, both count
            failed.append((pin.__name__, type(e).__name__))
    return failed


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, "mutation anchor not found exactly once: %r" % old
    path = tmp_path / ("mut_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = oracle.build_variant(str(path), str(tmp_path / ("mut_%s.so" % name)))
    with oracle.use_library(so):
        failed = _run_pins()
    assert failed, "planted mistake %s passed every pin" % name
