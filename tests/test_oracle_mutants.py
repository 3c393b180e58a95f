"""The pins must be strong enough to catch plausible mistakes.

Each case below plants one mistake (a dropped factor, a flipped sign, a
transposed operand, a wrong index, a missing correction) in a temporary copy
of the oracle's C source, builds it, and requires that at least one pin of
test_oracle_pins fails against it.  The real oracle is never modified.
"""
import os
import shutil
import subprocess

import pytest

import oracle.oracle as OO
from tests import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(OO.__file__), "efunc_oracle.c")
HDR = os.path.join(os.path.dirname(OO.__file__), "efunc_oracle.h")

MUTANTS = {
    "grad_c_drops_factor_2": ("-k[5] + 2.0 * k[3] * x0 * r, -k[6]", "-k[5] + k[3] * x0 * r, -k[6]"),
    "grad_beta_sign": ("dl * w * (-x2n) * r", "dl * w * (x2n) * r"),
    "value_transposed_slope": ("(q[1] - a[1]) * a[6] + (q[2]", "(q[1] - a[1]) * a[5] + (q[2]"),
    "logit_wrong_index": ("z = q[2] - a[2];\n    return -a[3]", "z = q[2] - a[1];\n    return -a[3]"),
    "rho_chain_rule_missing": ("t[4] = g->raw_beta ? a[3] : exp((double)p[4]) * a[3];", "t[4] = a[3];"),
    "adam_no_bias_correction": ("const double mh = m[i] / bc1", "const double mh = m[i]"),
    "meanshift_no_minus_k": ("delta[3 * i + 1] = sy / w - k[1];", "delta[3 * i + 1] = sy / w;"),
    "offset_sign": ("b[1] = ky + (double)p[6];", "b[1] = ky - (double)p[6];"),
    "lse_drops_max": ("*lse = M + log(e);", "*lse = log(e);"),
    "truncation_too_tight": ("if (s >= t->M - t->T) {", "if (s >= t->M - 0.5 * t->T) {"),
    # the tolerance scales every parity check rests on
    "sigma_not_normalised": ("*sigma = sa / e;", "*sigma = sa;"),
    "trunc_sigma_x10": ("if (sigma) sigma[j] = t.sa / t.e;", "if (sigma) sigma[j] = 10.0 * t.sa / t.e;"),
    "grad_scale_x10": ("const double adw = fabs(dl) * w;", "const double adw = 10.0 * fabs(dl) * w;"),
    "trunc_grad_scale_x10": ("adw = fabs(dLdO[j]) * w;", "adw = 10.0 * fabs(dLdO[j]) * w;"),
    "grad_scale_beta_drops_r": ("adw * x2n * fabs(r),", "adw * x2n,"),
    "kappa_x100": ("k += wr * fabs(s);", "k += 100.0 * wr * fabs(s);"),
    "tail_x10": ("if (s - lse < -T) tl += wr;", "if (s - lse < -T) tl += 10.0 * wr;"),
    "subthreshold_wrong_side": ("const int below = lw < -T;", "const int below = lw > -T;"),
    "qsig_drops_factor_2": ("const double bxa = 2.0 * k[3] * w * fabs(x);",
                            "const double bxa = k[3] * w * fabs(x);"),
    "qkap_x100": ("qk[d] += w * fabs(s) * fabs(ga - G[d])", "qk[d] += 100.0 * w * fabs(s) * fabs(ga - G[d])"),
    "qkap_drops_value_errors": ("qk[d] += w * fabs(s) * fabs(ga - G[d]) + bxa * sa;",
                                "qk[d] += w * fabs(s) * fabs(ga - G[d]);"),
    "qbx_drops_abs": ("const double bxa = 2.0 * k[3] * w * fabs(x);\n                qs[d]",
                      "const double bxa = 2.0 * k[3] * w * x;\n                qs[d]"),
    "qtail_drops_renormalisation": ("if (below) qt[d] += w * (fabs(ga) + fabs(G[d]));",
                                    "if (below) qt[d] += w * fabs(ga);"),
    "trunc_band_wrong_side": ("if (bk && s - lse[j] < -Tb) {", "if (bk && s - lse[j] > -Tb) {"),
    "trunc_band_from_max": ("if (bk && s - lse[j] < -Tb) {", "if (bk && s - M[j] < -Tb) {"),
    "trunc_band_search_too_short": ("const double Tr = (bk && T2 > T) ? T2 : T;", "const double Tr = T;"),
}

PINS = [getattr(P, n) for n in dir(P) if n.startswith("test_")]


def _run_pins(orc):
    failures = []
    for fn in PINS:
        params = getattr(fn, "pytestmark", [])
        kwargs_list = [{}]
        for mk in params:
            if mk.name == "parametrize":
                name, vals = mk.args
                kwargs_list = [{name: v} for v in vals]
        for kw in kwargs_list:
            try:
                fn(orc, **kw)
            except AssertionError:
                failures.append(fn.__name__)
                return failures
            except Exception:  # noqa: BLE001 - a crash also counts as caught
                failures.append(fn.__name__ + " (error)")
                return failures
    return failures


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, orc):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {name}"
    shutil.copy(HDR, tmp_path / "efunc_oracle.h")
    (tmp_path / "efunc_oracle.c").write_text(src.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", lib,
                           str(tmp_path / "efunc_oracle.c"), "-lm"])
    with OO.use_library(lib):
        caught = _run_pins(orc)
    assert caught, f"no pin caught mutant {name}"
