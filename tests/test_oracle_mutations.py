"""Planted mistakes in the oracle, one at a time, each of which the oracle's
pins must catch (opt-in: CTMHD_MUTATION_TESTS=1; from a second to about
100 s per case, about ten minutes for all sixteen on 8 cores).

Each case edits one expression of a copy of oracle/ctmhd_oracle.cpp (a sign,
an index, an operand, a dropped term), builds it as the oracle library and
runs the CPU pins (tests/test_oracle_units.py, tests/test_oracle_step.py)
against it through CTMHD_ORACLE_LIB: the run must fail.  Everything happens
on the CPU; the HIP path is not involved."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ctmhd_oracle.cpp")

# name: (expression in the oracle, planted mistake)
MUTATIONS = {
    "ld04_sign": ("                apb * amb / (apb + amb) * (baT - baB) + apa",
                  "                apb * amb / (apb + amb) * (baT - baB) - apa"),
    "hlld_double_star_energy_sign": ("R essL = esL - sqL * (vbsL - vbss) * sg;",
                                     "R essL = esL + sqL * (vbsL - vbss) * sg;"),
    "q26_corner_operand": ("eps[1] = -uaB * bbR + ubR * baB;", "eps[1] = -uaB * bbR + ubL * baB;"),
    "edge_alpha_not_max": ("R apa = rmax(FD.ap[a][fa0], FD.ap[a][fa1]);", "R apa = FD.ap[a][fa1];"),
    "ppm_interface_weight": ("return R(0.5) * (qb + qc) - (dmc - dmb) / R(6.0);",
                             "return R(0.5) * (qb + qc) - (dmc - dmb) / R(3.0);"),
    "joule_sign": ("F[a][4][f] = F[a][4][f] + (eb * bc - ec * bb);",
                   "F[a][4][f] = F[a][4][f] + (eb * bc + ec * bb);"),
    "resistive_emf_sign": ("            e = e + R(P.eta) * jc;", "            e = e - R(P.eta) * jc;"),
    "hlld_star_field": ("R f = (s.rho * d * d - bn2) / q;", "R f = (s.rho * d * dsm - bn2) / q;"),
    "q26_face_velocity_weights": (
        "FD.us[a][f] = (apv * sL.un + amv * sR.un) / (apv + amv);",
        "FD.us[a][f] = (amv * sL.un + apv * sR.un) / (apv + amv);"),
    "b25a_reconstruction_order": (
        "R e_ba = recon_two_step(g, recon, ecell, p, b, a, sb, sa);",
        "R e_ba = recon_two_step(g, recon, ecell, p, b, a, sa, sb);"),
    "rk2_average": ("S.c[m][x] = Sn.c[m][x] + R(0.5) * (D1S[m][x] + D2S[m][x]);",
                    "S.c[m][x] = Sn.c[m][x] + R(0.5) * (D1S[m][x] + D1S[m][x]);"),
    "no_hll_fallback": ("if (bad) { hll(UL, FL, UR, FR, SL, SR, F); return 1; }",
                        "if (false) { hll(UL, FL, UR, FR, SL, SR, F); return 1; }"),
    "fs18_order_side": (
        "recon_two_step(g, recon, W.u[a], p, b, a, sb, sa));",
        "recon_two_step(g, recon, W.u[a], p, b, a, sa, sb));"),
    "fs18_face_field_side": ("R bbX = sa == 0 ? bbL : bbR;", "R bbX = sa == 0 ? bbR : bbL;"),
    "dual_quotient_rule": ("return {q, (a.d - q * b.d) / b.v};",
                           "return {q, (a.d + q * b.d) / b.v};"),
    "fofc_edge_rule": (
        "if (flag[c] || flag[g.idx(q1.v)] || flag[g.idx(q2.v)] || flag[g.idx(q3.v)]) {",
        "if (flag[c] || flag[g.idx(q1.v)] || flag[g.idx(q2.v)]) {"),
}

pytestmark = pytest.mark.skipif(os.environ.get("CTMHD_MUTATION_TESTS") != "1",
                                reason="opt-in: set CTMHD_MUTATION_TESTS=1")


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    good, bad = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(good) == 1, "the expression to mutate is no longer in the oracle"
    cpp = tmp_path / "mutant.cpp"
    cpp.write_text(src.replace(good, bad))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-o", str(lib), str(cpp)])
    env = dict(os.environ, CTMHD_ORACLE_LIB=str(lib), CTMHD_MUTATION_TESTS="0")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_oracle_units.py"),
                        os.path.join(ROOT, "tests", "test_oracle_step.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1800)
    print(name, [ln for ln in r.stdout.splitlines() if "FAILED" in ln or "passed" in ln][:3])
    assert r.returncode != 0, f"planted mistake {name} passed every pin"
