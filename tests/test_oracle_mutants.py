"""Planted mistakes: each one is a plausible slip in the oracle (a dropped term,
a wrong sign, weight or index), planted in a temporary copy of ``oracle.c``
on the CPU. The pins must catch every one of them, otherwise they are not
strong enough to trust the oracle.
"""
import pytest

import adjoint_pins
import fd4_pins
import generic_pins
import oracle
import pins

MUTANTS = {
    "rest weight": ("W[5] = {1.0 / 3.0, 1.0 / 6.0,", "W[5] = {1.0 / 6.0, 1.0 / 6.0,"),
    "one link weight": ("1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};", "1.0 / 6.0, 1.0 / 6.0, 1.0 / 3.0};"),
    "tau without c_s^2": ("return 0.5 + d_lattice / CS2;", "return 0.5 + d_lattice;"),
    "relaxation factor tau-1/2": ("(tau[c] - 1.0) * (rho_f", "(tau[c] - 0.5) * (rho_f"),
    "centre weight in the bracket": ("rho_f - 2.0 * rho_c + rho_b", "rho_f - rho_c + rho_b"),
    "start from centre not rho_b": ("rho_b + (tau[c] - 1.0)", "rho_c + (tau[c] - 1.0)"),
    "N instead of N_c": ("double Nc = S + E + I + R;", "double Nc = S + E + I + R + rho[CD];"),
    "no incubation outflow": ("psi[CE] = force - k.alpha * E;", "psi[CE] = force;"),
    "removal scaled by phi": ("psi[CI] = k.alpha * E - k.gamma * I;",
                              "psi[CI] = k.alpha * E - k.gamma * k.phi * I;"),
    "recovery uses phi": ("psi[CR] = (1.0 - k.phi) * k.gamma * I;",
                          "psi[CR] = k.phi * k.gamma * I;"),
    "deaths from E": ("psi[CD] = k.phi * k.gamma * I;", "psi[CD] = k.phi * k.gamma * E;"),
    "no guard on N_c": ("    if (Nc > 0.0)\n        force", "    if (1)\n        force"),
    "guard admits N_c = 0": ("    if (Nc > 0.0)\n        force", "    if (Nc >= 0.0)\n        force"),
    "force not divided by N_c": ("force = k.beta * S * I / Nc;", "force = k.beta * S * I;"),
    "force uses E": ("force = k.beta * S * I / Nc;", "force = k.beta * S * E / Nc;"),
    "no-flux ghost zero": ("return field[(size_t)yc * nx + xc];", "return 0.0;"),
    "periodic wrap off by one": ("x = ((x % nx) + nx) % nx;", "x = ((x % nx) + nx + 1) % nx;"),
    "source without dt": ("+ psi[c] * dt;", "+ psi[c];"),
    "deceased ODE from wrong source": ("centre[CD] + psi[CD] * dt;", "centre[CD] + psi[CI] * dt;"),
    "wrong link vector": ("CY[5] = {0, 0, 1, 0, -1};", "CY[5] = {0, 0, 1, 0, 1};"),
    "BGK relaxation times tau": ("f + (feq - f) / tau[c] +", "f + (feq - f) * tau[c] +"),
    "BGK source without weight": ("+ W[i] * psi[c] * dt;", "+ psi[c] * dt;"),
    "BGK bounce-back same direction": ("f_out[fidx(c, OPP[i], plane) + cell] = fstar;",
                                       "f_out[fidx(c, i, plane) + cell] = fstar;"),
    "BGK density drops a population": ("s += f_in[fidx(c, i, plane) + cell];",
                                       "s += (i < 4) ? f_in[fidx(c, i, plane) + cell] : 0.0;"),
    "BGK deceased frozen": ("rhoD_out[cell] = rho[CD] + psi[CD] * dt;",
                            "rhoD_out[cell] = rho[CD];"),
    "BGK equilibrium from f": ("double feq = W[i] * rho[c];", "double feq = W[i] * f;"),
    "BGK opposite table": ("OPP[5] = {0, 3, 4, 1, 2};", "OPP[5] = {0, 4, 3, 2, 1};"),
    "adjoint back-read weight": ("back[nb_b] += lam[c] * W[i] * tau[c];",
                                 "back[nb_b] += lam[c] * W[i] * (tau[c] - 0.5);"),
    "adjoint centre sign": ("lam[c] * (-2.0) * (tau[c] - 1.0)", "lam[c] * 2.0 * (tau[c] - 1.0)"),
    "adjoint resting deceased dropped": ("back[cell] += lam[c];\n", "back[cell] += 0.0;\n"),
    "adjoint no-flux ghost to node 0": ("size_t nb_b = cell, nb_f = cell;",
                                        "size_t nb_b = 0, nb_f = 0;"),
    "adjoint periodic wrap": ("nb_f = (size_t)(((yf % ny) + ny) % ny) * nx + ((xf % nx) + nx) % nx;",
                              "nb_f = (size_t)(((yf % ny) + ny) % ny) * nx + ((xf % nx) + nx + 1) % nx;"),
    "adjoint dF/dS without -F/N": ("double fS = k.beta * I / Nc - F / Nc;",
                                   "double fS = k.beta * I / Nc;"),
    "adjoint dF/dE zero": ("double fE = -F / Nc;", "double fE = 0.0;"),
    "adjoint dF/dR zero": ("double fR = -F / Nc;", "double fR = 0.0;"),
    "adjoint incubation sign": ("(lI - lE) * k.alpha * dt;", "(lE - lI) * k.alpha * dt;"),
    "adjoint deaths without phi": ("k.phi * lD) * k.gamma * dt;", "lD) * k.gamma * dt;"),
    "adjoint beta gradient not over N_c": ("grad[0] += (lE - lS) * dt * S * I / Nc;",
                                           "grad[0] += (lE - lS) * dt * S * I;"),
    "adjoint alpha gradient from I": ("grad[1] += (lI - lE) * E * dt;",
                                      "grad[1] += (lI - lE) * I * dt;"),
    "adjoint gamma gradient from E": ("k.phi * lD) * I * dt;", "k.phi * lD) * E * dt;"),
    "adjoint phi gradient sign": ("grad[3] += (lD - lR) * k.gamma * I * dt;",
                                  "grad[3] += (lR - lD) * k.gamma * I * dt;"),
    "adjoint d gradient without c_s^2": ("* 3.0 * dt / (dx * dx);", "* dt / (dx * dx);"),
    "D2Q9 diagonal weight": ("1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};",
                             "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 18.0};"),
    "D2Q9 diagonal vector": ("CX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};",
                             "CX9[9] = {0, 1, 0, -1, 0, 1, 1, -1, 1};"),
    "generic catalyst ignored": ("                    flow *= centre[cat[r]];",
                                 "                    flow *= 1.0;"),
    "generic frequency ignored": ("                if (freq[r])\n", "                if (0)\n"),
    "generic half outflow": ("psi[src[r]] -= flow;", "psi[src[r]] -= 0.5 * flow;"),
    "generic counts every compartment": ("                if (counted[c])\n",
                                         "                if (1)\n"),
    "D2Q9 mirror off by one": ("x = 2 * nx - 1 - x;", "x = 2 * nx - 2 - x;"),
    "D2Q9 mirror of y": ("y = -1 - y;", "y = -y;"),
    "FD4 outer weight sign": ("- u[(size_t)y * nx + fd4_fold(x + 2, nx, bc)];",
                              "+ u[(size_t)y * nx + fd4_fold(x + 2, nx, bc)];"),
    "FD4 centre weight in y": ("- 30.0 * here[c]\n                                 + 16.0 * u[(size_t)fd4_fold(y + 1",
                               "- 28.0 * here[c]\n                                 + 16.0 * u[(size_t)fd4_fold(y + 1"),
    "FD4 without the 1/12": ("double h2 = 12.0 * dx * dx;", "double h2 = dx * dx;"),
    "FD4 far neighbour on the wrong side": ("-u[(size_t)y * nx + fd4_fold(x - 2, nx, bc)]",
                                            "-u[(size_t)y * nx + fd4_fold(x + 2, nx, bc)]"),
    "FD4 periodic wrap off by one": ("return ((i % n) + n) % n;", "return ((i % n) + n + 1) % n;"),
    "FD4 reflection about the node": ("return m < n ? m : period - 1 - m;",
                                      "return m < n ? m : (period - 1 - m + 1) % n;"),
    "FD4 diffusivity of S for all": ("F[c * plane + cell] = d[c] * (along_x",
                                     "F[c * plane + cell] = d[0] * (along_x"),
    "RK4 second stage from k1": ("stage[i] = rho[i] + 0.5 * dt * k2[i];",
                                 "stage[i] = rho[i] + 0.5 * dt * k1[i];"),
    "RK4 third stage half step": ("stage[i] = rho[i] + dt * k3[i];",
                                  "stage[i] = rho[i] + 0.5 * dt * k3[i];"),
    "RK4 weights": ("(k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i])",
                    "(k1[i] + 2.0 * k2[i] + k3[i] + 2.0 * k4[i])"),
    "FD4 reactions left out": ("(along_x + along_y) / h2 + psi[c];", "(along_x + along_y) / h2;"),
}


def _caught(orc) -> list:
    failures = []
    for check in (pins.FAST_SSLBM_CHECKS + pins.FAST_BGK_CHECKS + adjoint_pins.FAST_ADJOINT_CHECKS
                  + generic_pins.FAST_GENERIC_CHECKS + fd4_pins.FAST_FD4_CHECKS):
        try:
            check(orc)
        except (AssertionError, ValueError, FloatingPointError) as exc:
            failures.append(f"{check.__name__}: {str(exc)[:80]}")
    return failures


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    original, mutated = MUTANTS[name]
    source = oracle.SOURCE.read_text()
    assert source.count(original) == 1, f"mutation site for '{name}' not unique in oracle.c"
    src = tmp_path / "oracle_mutant.c"
    src.write_text(source.replace(original, mutated))
    lib = oracle.compile_library(src, tmp_path / "liboracle_mutant.so")
    failures = _caught(oracle.Oracle(lib))
    assert failures, f"planted mistake '{name}' passed every pin"
