"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (on the CPU), builds it, and runs
the pin tests against that build: they must fail. A case whose mutant passes every pin names a
part of the oracle that nothing outside it checks.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sfhk_oracle.c")
HDR = os.path.join(ROOT, "oracle", "sfhk_oracle.h")
PINS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
        os.path.join(ROOT, "tests", "test_oracle_sfa.py")]

MUTANTS = {
    "G imaginary part sign": ("G[i][k].im = fma(M_PQ(m, i, k), inv4g, -(gamma * M_QP(m, i, k)));",
                              "G[i][k].im = -fma(M_PQ(m, i, k), inv4g, -(gamma * M_QP(m, i, k)));"),
    "1/(2 gamma) for 1/(4 gamma)": ("double inv4g = 1.0 / (4.0 * gamma);",
                                    "double inv4g = 1.0 / (2.0 * gamma);"),
    "gamma dq/dp0 term doubled": ("-(gamma * M_QP(m, i, k))", "-(2.0 * gamma * M_QP(m, i, k))"),
    "Hessian force sign": ("kP[i] = -t;", "kP[i] = t;"),
    "field table: sign of the envelope term": ("e_half[m] = a - b;", "e_half[m] = a + b;"),
    "field table: envelope frequency doubled": ("traj_sincos((M_PI * t) / T, &s1, &c1);",
                                                "traj_sincos((2.0 * M_PI * t) / T, &s1, &c1);"),
    "field dropped from the action": ("L = fma(-q[2], E, L);", "L = L;"),
    "field force sign": ("k[5] = -fma(g, q[2], E);", "k[5] = -fma(g, q[2], -E);"),
    "RK4 weight of k3": ("acc = fma(2.0, k3[i], acc);", "acc = acc + k3[i];"),
    "RK4 stage-3 time": ("rhs(pot, eb, ys, k3);", "rhs(pot, ea, ys, k3);"),
    "overlap phase conjugated": ("(gamma * q2 + I * pq)) / (4.0 * ga);\n    if (creal(ex) < -cut) continue; /* primitive",
                                 "(gamma * q2 - I * pq)) / (4.0 * ga);\n    if (creal(ex) < -cut) continue; /* primitive"),
    "velocity: exponent phase conjugated": ("(gamma * q2 + I * pq)) / (4.0 * ga);\n    if (creal(ex) < -cut) continue; /* the dipole",
                                            "(gamma * q2 - I * pq)) / (4.0 * ga);\n    if (creal(ex) < -cut) continue; /* the dipole"),
    "overlap s-wave power": ("coef[j] * pow(ga, -2.5)", "coef[j] * pow(ga, -1.5)"),
    "overlap p-wave bracket": ("(a * a + 2.0 * ga)", "(a * a + ga)"),
    "no branch tracking": ("if (sgn * dot < 0.0) sgn = -sgn;", ""),
    "screened V' drops Z'": ("double vp = fma(Z * r, ir3, d1 * ir);", "double vp = Z * r * ir3;"),
    "screened V'' factor": ("double vpp = tc - fma(2.0, tb, ta);", "double vpp = tc - fma(1.0, tb, ta);"),
    "softcore Hessian factor": ("*c = (-3.0 * Z) * u5;", "*c = (-2.0 * Z) * u5;"),
    "Kay test on |det|^2": ("if (!(a2 <= kay2) || !finite)", "if (!(a2 <= hk->kay_max) || !finite)"),
    "birth ties to upper": ("double n = ceil(u - 0.5);", "double n = floor(u + 0.5);"),
    "dipole sign": ("d_out[n] = -2.0 * f[n];", "d_out[n] = 2.0 * f[n];"),
    "Hann window sign": ("0.5 * (1.0 + cos(M_PI * t / tau_h))", "0.5 * (1.0 - cos(M_PI * t / tau_h))"),
    "resample neighbour": ("d[i] + frac * (d[i + 1] - d[i])", "d[i] + frac * (d[i] - d[i])"),
    "Ip phase sign": ("* o * cexp(I * (y[IY_S] - gs->ip * tn))", "* o * cexp(I * (y[IY_S] + gs->ip * tn))"),
    "default weight sign": ("return cexp(I * pq) / (double)n;", "return cexp(-I * pq) / (double)n;"),
    "exp reference not correctly rounded": ("return (double)expq((__float128)x);",
                                            "return (double)(float)expq((__float128)x);"),
    "contract exp drops the ln2 tail": ("r = fma(-k, EXPC_LN2_LO, r);", "r = r;"),
    "contract exp one degree short": ("double p = inv_fact[13];\n  for (int n = 12;",
                                      "double p = inv_fact[12];\n  for (int n = 11;"),
    "screened exponent scale": ("-(r / pot->r_scr) : -(r * inv_rs));",
                                "-(r / pot->r_scr) : -(r * inv_rs * 0.5));"),
    "screened 1/r^2 in the Hessian": ("*c = (vpp - *g) * (inv_r * inv_r);",
                                      "*c = (vpp - *g) * inv_r;"),
    "rsqrt: one Newton step short": ("for (int it = 0; it < 3; ++it)", "for (int it = 0; it < 2; ++it)"),
    "rsqrt: tiny arguments unscaled": ("return rsqrt_core(x * 0x1p1000) * 0x1p500;",
                                       "return rsqrt_core(x);"),
    "principal sqrt: imaginary part halved twice": ("(0.5 * z.im) / t : (0.5 * z.im) * rw;",
                                                    "(0.5 * z.im) / t : (0.25 * z.im) * rw;"),
    "SFA: crossing sign ignored in the bisection": ("if ((up ? v : -v) < kap)", "if (v < kap)"),
    "SFA: Newton derivative without w_m": ("*dv = -(a->K * (a->C[0] * a->om[0] * ch[0] +",
                                           "*dv = -(a->K * (a->C[0] * ch[0] +"),
    "SFA: Newton step sign": ("double tn = t - f / fp;", "double tn = t + f / fp;"),
    "SFA: tunnel exit sign": ("*qz = -(a.K * (a.C[0]", "*qz = (a.K * (a.C[0]"),
    "SFA: k_z from sinh instead of cosh - 1": ("double c0 = coshm1_c(a.om[0] * t);",
                                              "double c0 = sinh_c(a.om[0] * t);"),
    "SFA: sinh as cosh": ("return 0.5 * (e - 1.0 / e);", "return 0.5 * (e + 1.0 / e);"),
    "SFA: envelope sideband frequency": ("a->om[1] = pl->omega + W;", "a->om[1] = pl->omega + 2.0 * W;"),
    "SFA: action under the barrier sign": ("double complex S = gs->ip * ts + I * integ;",
                                           "double complex S = gs->ip * ts - I * integ;"),
    "SFA: modified weight without 1/(E.k)": ("amp = cexp(I * S) / ek;", "amp = cexp(I * S);"),
    "SFA: s-wave tunnelling element phase": ("-I * (0.5 * pow(M_PI, 1.5)) * kzs * sum",
                                             "(0.5 * pow(M_PI, 1.5)) * kzs * sum"),
    "SFA: p-wave tunnelling bracket": ("(2.0 * al - kzs * kzs) * e;", "(al - kzs * kzs) * e;"),
    "SFA: weight without e^{i p0.q0}": ("wj = u * cexp(I * (kz * qz)) * amp;", "wj = u * amp;"),
    "velocity: s-wave constant": ("return gs->l == 0 ? 2.0 * b * sum : 4.0 * I * gamma * sum;",
                                  "return gs->l == 0 ? b * sum : 4.0 * I * gamma * sum;"),
    "velocity: p-wave phase": ("return gs->l == 0 ? 2.0 * b * sum : 4.0 * I * gamma * sum;",
                               "return gs->l == 0 ? 2.0 * b * sum : 4.0 * gamma * sum;"),
    "velocity: q_z term sign": ("double complex b = p[2] - 2.0 * I * gamma * q[2];",
                                "double complex b = p[2] + 2.0 * I * gamma * q[2];"),
    "velocity: p-wave bracket": ("(b * b / (2.0 * gamma) + ga / al)", "(b * b / (2.0 * gamma) + 1.0)"),
    "velocity: Ip phase sign": ("ov * cexp(I * (y[IY_S] - gs->ip * tn));",
                                "ov * cexp(I * (y[IY_S] + gs->ip * tn));"),
    "velocity: alpha factor dropped (s)": ("sum += gs->coef[j] * al * pow(ga, -2.5) * cexp(ex);",
                                           "sum += gs->coef[j] * pow(ga, -2.5) * cexp(ex);"),
    "partial waves: band edges shifted": ("while (k < 7 && !(l2 < (k + 0.5) * (k + 0.5))) ++k;",
                                          "while (k < 7 && !(l2 < (k + 1.0) * (k + 1.0))) ++k;"),
    "partial waves: radius not squared": ("if (!(r2 < hk->pw_radius * hk->pw_radius))",
                                          "if (!(r2 < hk->pw_radius))"),
    "partial waves: cross product component": ("double cy = fma(q[2], p[0], -(q[0] * p[2]));",
                                               "double cy = fma(q[2], p[0], q[0] * p[2]);"),
    "partial waves: far bit ignored": ("return (hk->pw_mask >> 8) & 1;", "return 0;"),
    "gabor: window width": ("win[i] = exp(-0.5 * u * u);", "win[i] = exp(-u * u);"),
    "gabor: phase sign": ("cexp(I * (w * (t_first + (double)i * dt)))",
                          "cexp(-I * (w * (t_first + (double)i * dt)))"),
    "gabor: centre grid": ("double tc = tc_first + (double)c * tc_step;",
                           "double tc = tc_first + (double)(c + 1) * tc_step;"),
    "gabor: missing dt": ("    acc *= dt;\n", "\n"),
    "sincos: quadrant 1 cosine sign": ("case 1: *s = cr; *c = -sr; break;",
                                       "case 1: *s = cr; *c = sr; break;"),
    "sincos: reduction drops the pi/2 tail": ("r = fma(-k, SINC_PIO2_3, r);", "r = r;"),
    "sincos: sine series two terms short": ("double ps = inv_fact[17];\n  for (int j = 7;",
                                            "double ps = inv_fact[13];\n  for (int j = 5;"),
    "skip rule: threshold a quarter of the cut": ("if (creal(ex) < -cut) continue; /* primitive negligible",
                                                  "if (creal(ex) < -0.25 * cut) continue; /* primitive negligible"),
    "skip rule: comparison inverted": ("if (creal(ex) < -cut) continue; /* primitive negligible",
                                       "if (creal(ex) >= -cut) continue; /* primitive negligible"),
    "velocity skip rule: threshold a quarter of the cut": ("if (creal(ex) < -cut) continue; /* the dipole",
                                                           "if (creal(ex) < -0.25 * cut) continue; /* the dipole"),
    "Kay whole-removal reading ignored": ("if (to.death < 0) run_traj(", "run_traj("),
    "velocity skip rule: comparison inverted": ("if (creal(ex) < -cut) continue; /* the dipole",
                                                "if (creal(ex) >= -cut) continue; /* the dipole"),
}


def _run_mutant(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: snippet not found exactly once"
    d = os.path.join(tmp, name.replace(" ", "_").replace("/", "_").replace("'", ""))
    os.makedirs(d, exist_ok=True)
    open(os.path.join(d, "sfhk_oracle.c"), "w").write(src.replace(old, new))
    open(os.path.join(d, "sfhk_oracle.h"), "w").write(open(HDR).read())
    lib = os.path.join(d, "libmut.so")
    subprocess.run(["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fPIC", "-shared",
                    "-std=gnu11", "-w", "-o", lib, os.path.join(d, "sfhk_oracle.c"),
                    "-lquadmath", "-lm", "-lpthread"], check=True)
    env = dict(os.environ, SFHK_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-x", "-q", "-p", "no:cacheprovider",
                        "-W", "ignore"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            futs = [ex.submit(_run_mutant, n, o, w, tmp) for n, (o, w) in MUTANTS.items()]
            results = dict(f.result() for f in futs)
    survivors = [n for n, rc in results.items() if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"
