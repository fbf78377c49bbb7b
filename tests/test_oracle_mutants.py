"""The pins must catch plausible mistakes in the oracle.  Each case plants one
mistake in a copy of oracle/lattice_oracle.c (a dropped or wrong term, a sign,
an index, a coefficient), builds it with gcc into a temporary library and runs
the named pins against it in a subprocess: at least one of them must fail."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lattice_oracle.c")

MUTANTS = [
    ("laplacian centre weight", "f[nbr(N, x, y, z, d, +1)] - 2.0 * f0 + f[nbr(N, x, y, z, d, -1)]",
     "f[nbr(N, x, y, z, d, +1)] - 3.0 * f0 + f[nbr(N, x, y, z, d, -1)]", "test_oracle_scalar.py"),
    ("potential force sign", "out[n] = c1 * lap[n] - c3 * pot_deriv(p, s, phi[0][n], chi);",
     "out[n] = c1 * lap[n] + c3 * pot_deriv(p, s, phi[0][n], chi);", "test_oracle_scalar.py"),
    ("Friedmann kinetic weight", "((al - 2.0) * EK_tot(E)", "((al - 1.0) * EK_tot(E)", "test_oracle_scalar.py"),
    ("drift scale factor", "drift(st, a_mid, h);                                          /* phi drift      */",
     "drift(st, a_n1, h);", "test_oracle_scalar.py"),
    ("Yoshida middle weight sign", "*w0 = -c / (2.0 - c);", "*w0 = c / (2.0 - c);", "test_oracle_scalar.py"),
    ("triple-jump exponent", "double c = pow(2.0, 1.0 / (double)(n + 1));", "double c = pow(2.0, 1.0 / (double)(n + 2));",
     "test_oracle_scalar.py"),
    ("Yoshida composition in reverse order",
     "            w[i] = y[m - 1 - i];          /* outermost first */\n            w[2 * m - i] = y[m - 1 - i];",
     "            w[i] = y[i];\n            w[2 * m - i] = y[i];", "test_oracle_scalar.py"),
    ("Yoshida central weight without the factor 2", "w[m] = 1.0 - 2.0 * sum;", "w[m] = 1.0 - sum;",
     "test_oracle_scalar.py"),
    ("leapfrog first half kick", "double w = (c->lf_stag == 0) ? 0.5 * h : h;", "double w = h;",
     "test_oracle_scalar.py"),
    ("leapfrog b kick without the kinetic average",
     "st.b += 0.5 * h * kernel_a(p, st.a, &Eb) + 0.5 * h * kernel_a(p, st.a, &Ea);",
     "st.b += h * kernel_a(p, st.a, &Ea);", "test_oracle_lf_self.py"),
    ("leapfrog drift at the new scale factor", "drift(&st, 0.5 * (st.a + a_n1), h);", "drift(&st, a_n1, h);",
     "test_oracle_lf_self.py"),
    ("leapfrog half kick of b with the synchronised momenta",
     "st.b += w * kernel_a(p, st.a, &Ea);", "st.b += w * kernel_a(p, st.a, &Eb);", "test_oracle_lf_self.py"),
    ("leapfrog sync of b without the kinetic energy",
     "        energies E = energies_of(p, st.phi, st.pi, c->a);\n        c->b += w * kernel_a(p, c->a, &E);",
     "        energies E = energies_of(p, st.phi, st.pi, c->a);\n        E.EK[0] = E.EK[1] = 0.0;\n        c->b += w * kernel_a(p, c->a, &E);",
     "test_oracle_lf_self.py"),
    ("gradient energy power of a", "/ (double)V / (2.0 * a * a);", "/ (double)V / (2.0 * a);",
     "test_oracle_scalar.py"),
    ("U(1) current sign", "double J = e / dx * (pr * ai - pim * ar);", "double J = e / dx * (pr * ai + pim * ar);",
     "test_oracle_u1.py"),
    ("U(1) plaquette index", "A[i][nbr(N, x, y, z, j, +1)] +", "A[i][nbr(N, x, y, z, i, +1)] +",
     "test_oracle_u1.py"),
    ("U(1) backward link conjugation", "double cm = cos(e * dx * A[i][nm]), sm = sin(e * dx * A[i][nm]);",
     "double cm = cos(e * dx * A[i][nm]), sm = -sin(e * dx * A[i][nm]);", "test_oracle_u1.py"),
    ("U(1) magnetic force power of a", "cm_ = pow(a, p->alpha - 1.0);", "cm_ = pow(a, p->alpha + 1.0);",
     "test_oracle_u1_expansion.py"),
    ("U(1) link drift power of a", "ca = h * pow(a_mid, p->alpha - 1.0);", "ca = h * pow(a_mid, p->alpha - 3.0);",
     "test_oracle_u1_expansion.py"),
    ("U(1) current power of a", "FA[i][n] = cl * (p->kappa_g * J)", "FA[i][n] = cv * (p->kappa_g * J)",
     "test_oracle_u1_expansion.py"),
    ("U(1) electric energy power of a", "out[3] = nval(&ska) / (double)V / a4;", "out[3] = nval(&ska) / (double)V / a2;",
     "test_oracle_u1_expansion.py"),
    ("U(1) gauge weight in the b kernel", "(al - 1.0) * (E[3] + E[4])", "(al - 2.0) * (E[3] + E[4])",
     "test_oracle_u1_expansion.py"),
    ("U(1) leapfrog b kick without the kinetic average",
     "c->b += 0.5 * h * u1_kernel_a(p, c->a, Eb) + 0.5 * h * u1_kernel_a(p, c->a, Ea);",
     "c->b += h * u1_kernel_a(p, c->a, Ea);", "test_oracle_u1_expansion.py"),
    ("Hessian cross term", "double h01 = 2.0 * p->q * f * x;", "double h01 = p->q * f * x;",
     "test_oracle_adjoint.py"),
    ("spectrum shell normalisation", "v * v * v / (4.0 * ORC_PI * (double)b * b)", "v * v * v / (4.0 * ORC_PI * (double)b)",
     "test_oracle_spectrum.py"),
    ("spectrum shells by nearest radius",
     "long b = (long)sqrt((double)m);\n    while ((b + 1) * (b + 1) <= m) ++b;\n    while (b * b > m) --b;",
     "long b = (long)(sqrt((double)m) + 0.5);", "test_oracle_spectrum.py"),
    ("inverse DFT with the forward sign", "if (sign < 0) {", "if (sign != 0) {", "test_oracle_adjoint.py"),
    ("spectrum-bin gradient factor", "g[n] = 2.0 * cb * re[n];", "g[n] = cb * re[n];", "test_oracle_adjoint.py"),
    ("DFT over two axes only", "for (int axis = 0; axis < 3; ++axis) dft_axis", "for (int axis = 0; axis < 2; ++axis) dft_axis",
     "test_oracle_spectrum.py"),
    ("occupation Hubble term sign", "xr = cp * pr[i] + hub * fr[i]", "xr = cp * pr[i] - hub * fr[i]",
     "test_oracle_occupation.py"),
    ("occupation momentum power of a", "cp = pow(a, p->alpha - 3.0)", "cp = pow(a, p->alpha - 2.0)",
     "test_oracle_occupation.py"),
    ("occupation omega placement", "n[b] = pref * (om * sf[b] +", "n[b] = pref * (sf[b] / om +",
     "test_oracle_occupation.py"),
    ("occupation momentum weight with the inverse power of a",
     "pow(a, 2.0 * (1.0 - p->alpha)) * sx[b]", "pow(a, 2.0 * (p->alpha - 1.0)) * sx[b]",
     "test_oracle_occupation.py"),
    ("occupation momentum weight with half the power of a",
     "pow(a, 2.0 * (1.0 - p->alpha)) * sx[b]", "pow(a, 1.0 - p->alpha) * sx[b]", "test_oracle_occupation.py"),
    ("occupation momentum weight dropped", "pow(a, 2.0 * (1.0 - p->alpha)) * sx[b]", "sx[b]",
     "test_oracle_occupation.py"),
    ("occupation cross-coupling mass", "if (p->potential == ORC_PHI4_CHI2) d += p->q * w * w;", "",
     "test_oracle_occupation.py"),
    ("fixed-background adjoint drift at the kick time", "double dr = h * pow(am, al - 3.0);",
     "double dr = h * pow(a0, al - 3.0);", "test_oracle_adjoint.py"),
    ("fixed-background second adjoint kick at a_n", "jac_F_T(p, ph1, lpi, J, lap, kL1, kV1);",
     "jac_F_T(p, ph1, lpi, J, lap, kL0, kV0);", "test_oracle_adjoint.py"),
    ("coupling sensitivity without the potential factor", "*dq += 0.5 * h * kV1 * dot_dFdq(p, ph1, lpi);",
     "*dq += 0.5 * h * dot_dFdq(p, ph1, lpi);", "test_oracle_adjoint.py"),
    ("observable kinetic power of a", "ia6 = ia2 * ia2 * ia2;", "ia6 = ia2 * ia2;", "test_oracle_adjoint.py"),
    ("energy fraction of chi whatever the field", "double wX = s == f ? 1.0 : 0.0;", "double wX = s == 1 ? 1.0 : 0.0;",
     "test_oracle_adjoint.py"),
    ("self-consistent adjoint without the closing b kick", "double g6 = 0.5 * h * (*lb);", "double g6 = 0.0;",
     "test_oracle_adjoint_self.py"),
    ("self-consistent adjoint without the drift's scale-factor term", "    la1 += 0.5 * labar;\n", "",
     "test_oracle_adjoint_self.py"),
    ("scale-factor kernel derivative exponent", "return (2.0 * al + 1.0) * C * Q / a", "return (2.0 * al) * C * Q / a",
     "test_oracle_adjoint_self.py"),
    ("scale-factor kernel kinetic power of a", "gpi[s][n] += w * C * (al - 2.0) * pi[s][n] / (pow(a, 6.0)",
     "gpi[s][n] += w * C * (al - 2.0) * pi[s][n] / (pow(a, 4.0)", "test_oracle_adjoint_self.py"),
    ("a drift adjoint without h", "*lb += h * la1;", "*lb += la1;", "test_oracle_adjoint_self.py"),
    ("adjoint drift", "for (size_t n = 0; n < V; ++n) lpi[s][n] += dr * lphi[s][n];",
     "for (size_t n = 0; n < V; ++n) lpi[s][n] += 0.5 * dr * lphi[s][n];", "test_oracle_adjoint.py"),
    ("SU(2) magnetic force sign", "- cm_ * (2.0 / (g * dx * dx * dx) * vs[k]);",
     "+ cm_ * (2.0 / (g * dx * dx * dx) * vs[k]);", "test_oracle_su2.py"),
    ("SU(2) current without conjugation", "t += conj(psi[r]) * 0.5 * PAULI[k][r][s] * a[s];",
     "t += psi[r] * 0.5 * PAULI[k][r][s] * a[s];", "test_oracle_su2.py"),
    ("SU(2) lower staple without a dagger", "mat2 Sm = m2_mul(m2_mul(m2_dag(su2_link(U, j, nimj)),",
     "mat2 Sm = m2_mul(m2_mul(su2_link(U, j, nimj),", "test_oracle_su2.py"),
    ("SU(2) lower staple at the wrong site", "shift(N, cp, j, -1, cimj);", "shift(N, c, j, -1, cimj);",
     "test_oracle_su2.py"),
    ("SU(2) magnetic energy normalisation", "nadd(&sgb, 2.0 * mag /", "nadd(&sgb, mag /", "test_oracle_su2.py"),
    ("SU(2) link drift direction", "u[a] = sin(0.5 * th) * Ev[a] / len;", "u[a] = -sin(0.5 * th) * Ev[a] / len;",
     "test_oracle_su2.py"),
    ("SU(2) link drift on the right", "mat2 R = m2_mul(su2_exp(cu * p->g * p->dx, Ev), su2_link(U, i, n));",
     "mat2 R = m2_mul(su2_link(U, i, n), su2_exp(cu * p->g * p->dx, Ev));", "test_oracle_su2.py"),
    ("SU(2) Gauss transport the other way", "mat2 Y = m2_mul(m2_mul(m2_dag(Um), X), Um);",
     "mat2 Y = m2_mul(m2_mul(Um, X), m2_dag(Um));", "test_oracle_su2.py"),
    ("SU(2) backward link not conjugated", "m2_apply(m2_dag(su2_link(U, i, nm)), qm, b);",
     "m2_apply(su2_link(U, i, nm), qm, b);", "test_oracle_su2.py"),
    ("Gauss solve with the continuum Poisson symbol",
     "double sx = sin(ORC_PI * x / N), sy = sin(ORC_PI * y / N), sz = sin(ORC_PI * z / N);",
     "double sx = ORC_PI * x / N, sy = ORC_PI * y / N, sz = ORC_PI * z / N;", "test_oracle_gauss_init.py"),
    ("Gauss solve field as a backward difference", "E[i][n] = (re[nbr(N, x, y, z, i, +1)] - re[n]) / dx;",
     "E[i][n] = (re[n] - re[nbr(N, x, y, z, i, -1)]) / dx;", "test_oracle_gauss_init.py"),
    ("SU(2) initial charge without the 1/2 of T_a", "t += conj(psi[r]) * 0.5 * PAULI[a][r][q] * pp[q];",
     "t += conj(psi[r]) * PAULI[a][r][q] * pp[q];", "test_oracle_gauss_init.py"),
    ("SU(2) VV stages of the full step", "su2_vv2(p, phi, pi, U, E, c, t, w[i] * h);",
     "su2_vv2(p, phi, pi, U, E, c, t, h);", "test_oracle_gauge_vv.py"),
    ("U(1) VV stages without the time advance", "        u1_vv2(p, phi, pi, A, piA, c, t, w[i] * h);\n        t += w[i] * h;",
     "        u1_vv2(p, phi, pi, A, piA, c, t, w[i] * h);", "test_oracle_u1_expansion.py"),
    ("SU(2) plaquette order", "mat2 P = m2_mul(m2_mul(su2_link(U, i, n), su2_link(U, j, at(N, ci[0], ci[1], ci[2]))),",
     "mat2 P = m2_mul(m2_mul(su2_link(U, j, at(N, ci[0], ci[1], ci[2])), su2_link(U, i, n)),", "test_oracle_su2.py"),
    ("SU(2) staple force with a^{1+alpha}", "- cm_ * (2.0 / (g * dx * dx * dx) * vs[k]);",
     "- cl * (2.0 / (g * dx * dx * dx) * vs[k]);", "test_oracle_su2_expansion.py"),
    ("SU(2) current without a^{1+alpha}", "FE[3 * i + k][n] = cl * (g / dx * cimag(t))",
     "FE[3 * i + k][n] = (g / dx * cimag(t))", "test_oracle_su2_expansion.py"),
    ("SU(2) link drift without a^{alpha-1}", "cu = h * pow(a_mid, p->alpha - 1.0);", "cu = h;",
     "test_oracle_su2_expansion.py"),
    ("SU(2) electric energy over a^2", "out[3] = nval(&ske) / (double)V / a4;", "out[3] = nval(&ske) / (double)V / a2;",
     "test_oracle_su2_expansion.py"),
    ("SU(2) gauge energies in the b kernel with weight alpha",
     "static double su2_kernel_a(const orc_su2_params *p, double a, const double *E)\n{\n    double al = p->alpha;\n"
     "    return pow(a, 2.0 * al + 1.0) / 3.0 * p->kappa2 *\n"
     "           ((al - 2.0) * E[0] + al * E[1] + (al - 1.0) * (E[3] + E[4])",
     "static double su2_kernel_a(const orc_su2_params *p, double a, const double *E)\n{\n    double al = p->alpha;\n"
     "    return pow(a, 2.0 * al + 1.0) / 3.0 * p->kappa2 *\n"
     "           ((al - 2.0) * E[0] + al * E[1] + (al) * (E[3] + E[4])", "test_oracle_su2_expansion.py"),
    ("SU(2) leapfrog sync without the b half kick",
     "        su2_energy_plain(p, c->a, phi, pi, U, E, En);\n        c->b += w * su2_kernel_a(p, c->a, En);\n    }\n"
     "    su2_kick(p, c->a, phi, pi, U, E, w);\n    c->lf_stag = 0;",
     "        su2_energy_plain(p, c->a, phi, pi, U, E, En);\n    }\n"
     "    su2_kick(p, c->a, phi, pi, U, E, w);\n    c->lf_stag = 0;", "test_oracle_su2_expansion.py"),
]


@pytest.mark.parametrize("name,old,new,tests", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, tests):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mut.c")
        so = os.path.join(d, "libmut.so")
        open(c, "w").write(src.replace(old, new, 1))
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, c, "-lm"],
                       check=True, capture_output=True)
        env = dict(os.environ, ORACLE_LIB=so)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", tests)], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=600)
        assert r.returncode != 0, f"planted mistake '{name}' was not caught:\n{r.stdout[-2000:]}"
