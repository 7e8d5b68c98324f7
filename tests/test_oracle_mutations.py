"""Planted mistakes: every pin of the oracle must be able to fail.

Each case below copies the oracle's C source, plants one plausible mistake
in it (a dropped term, a wrong sign, factor, index or power of dx, a
transposed operand, an unwrapped angle, a shifted bit field), builds the
copy, and runs the pin suite (tests/test_oracle_pins.py) against it in a
separate process: at least one pin must fail.  A control build of the
unchanged source must pass, so a failure is the mistake's and not the
harness's.  CPU only; the mistakes live in temporary copies, never in the
oracle itself.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "ahref.c")

# (name, text in ahref.c, replacement); each text occurs exactly once
MUTATIONS = [
    ("link sign", "double s = -sin(dx * Aj);", "double s = sin(dx * Aj);"),
    ("conjugate link sign", "    double s = sin(dx * Aj);", "    double s = -sin(dx * Aj);"),
    ("alpha/2 -> alpha", "double delta = 0.5 * p->alpha * p->m * p->deta / eta;",
     "double delta = p->alpha * p->m * p->deta / eta;"),
    ("omega = delta", "out->omega = (1.0 - s) * delta;", "out->omega = delta;"),
    ("a without eta_ref", "double a = pow(eta / p->eta_ref, p->m);", "double a = pow(eta, p->m);"),
    ("potential without f", "double pot = 0.5 * p->lambda0 * sc->f *", "double pot = 0.5 * p->lambda0 *"),
    ("lambda/2 -> lambda/4", "double pot = 0.5 * p->lambda0", "double pot = 0.25 * p->lambda0"),
    ("current sign", "double J = (pr * wi - pim * wr) / dx;", "double J = (pim * wr - pr * wi) / dx;"),
    ("Laplacian power of dx", "    lr /= dx2;", "    lr /= dx;"),
    ("current without f", "fe[i] = -C + 2.0 * p->e0 * p->e0 * sc->f * J;", "fe[i] = -C + 2.0 * p->e0 * p->e0 * J;"),
    ("curl sign", "fe[i] = -C +", "fe[i] = C +"),
    ("transposed plaquette",
     "FLD(st, V, AA + i, y0) + FLD(st, V, AA + j, yi) - FLD(st, V, AA + i, yj) - FLD(st, V, AA + j, y0)",
     "FLD(st, V, AA + i, y0) + FLD(st, V, AA + j, yj) - FLD(st, V, AA + i, yi) - FLD(st, V, AA + j, y0)"),
    ("Pi damping with omega", "pi_out[c] = ((1.0 - sc->delta)", "pi_out[c] = ((1.0 - sc->omega)"),
    ("IC bit field", ">> 11) * 0x1.0p-53", ">> 12) * 0x1.0p-53"),
    ("unwrapped plaquette angle", "double thw = p->compact ? th - TWO_PI * rint(th / TWO_PI) : th;",
     "double thw = th;"),
    ("winding counted with sign", "acc[S_WABS] += (double)(w < 0 ? -w : w);", "acc[S_WABS] += (double)w;"),
    ("string length without dx", "out->L_W = p->dx * tot[S_WABS];", "out->L_W = tot[S_WABS];"),
    ("Gauss coupling without damping factor",
     "return 2.0 * p->e0 * p->e0 * sc.f * (1.0 + sc.delta) / (1.0 + sc.omega);",
     "return 2.0 * p->e0 * p->e0 * sc.f;"),
    ("uncentred momentum", "double pbr = 0.5 * (FLD(st, V, PIR, i0) + pin[0]);", "double pbr = FLD(st, V, PIR, i0);"),
    ("gauge energy factor", "double inv2e2f = 1.0 / (2.0 * p->e0 * p->e0 * sc->f);",
     "double inv2e2f = 1.0 / (p->e0 * p->e0 * sc->f);"),
    ("magnetic energy factor", "mag += p->compact ? 2.0 * (1.0 - cos(th)) / dx4",
     "mag += p->compact ? (1.0 - cos(th)) / dx4"),
    ("mu = pi sigma^2", "sqrt(-TWO_PI * p->sigma * p->sigma * vol / out->sum_L)",
     "sqrt(-0.5 * TWO_PI * p->sigma * p->sigma * vol / out->sum_L)"),
    ("box volume without dx", "double vol = pow((double)N * p->dx, 3.0);", "double vol = pow((double)N, 3.0);"),
    ("Gauss rms over N", "out->gauss_rms = sqrt(tot[S_G2] / (double)V);", "out->gauss_rms = sqrt(tot[S_G2] / (double)N);"),
    ("Gauss relative norm without charge", "double den = sqrt(tot[S_DIV2] + tot[S_CRHO2]);",
     "double den = sqrt(tot[S_DIV2]);"),
    ("unweighted R", "out->R = tot[S_KINL] / tot[S_GRADL];", "out->R = tot[S_KIN] / tot[S_GRAD];"),
    ("v2_phi factor", "out->v2_phi = 2.0 * out->R / (1.0 + out->R);", "out->v2_phi = out->R / (1.0 + out->R);"),
    ("v2_omega without 3", "out->v2_omega = 0.5 * (1.0 + 3.0 * tot[S_PL] / tot[S_RHOL]);",
     "out->v2_omega = 0.5 * (1.0 + tot[S_PL] / tot[S_RHOL]);"),
    ("gradient pressure sign", "double pres = kin - grad / 3.0 - pot + (el + mag) / 3.0;",
     "double pres = kin + grad / 3.0 - pot + (el + mag) / 3.0;"),
]

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def _build(src_text, out_dir, name):
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", *CFLAGS, "-I" + os.path.join(ROOT, "oracle"), c, "-o", so, "-lm"], check=True)
    return so


def _pins_pass(so) -> bool:
    env = dict(os.environ, AHREF_LIB=so, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode == 0


def test_planted_mistakes_fail_a_pin(tmp_path):
    src = open(SRC).read()
    for name, old, new in MUTATIONS:
        assert src.count(old) == 1, (name, src.count(old))
    builds = [("control", src)] + [(f"m{k:02d}", src.replace(old, new)) for k, (_, old, new) in enumerate(MUTATIONS)]
    sos = [_build(text, str(tmp_path), tag) for tag, text in builds]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        passed = list(ex.map(_pins_pass, sos))
    assert passed[0], "the unchanged oracle must pass its pins"
    survivors = [MUTATIONS[k][0] for k, ok in enumerate(passed[1:]) if ok]
    assert not survivors, f"planted mistakes that no pin catches: {survivors}"
