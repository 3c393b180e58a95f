"""The variant oracle's pins must catch plausible mistakes: each case plants
one in a temporary copy of efunc_oracle_var.c and requires that some pin of
test_oracle_var_pins fails against the mutant build."""
import os
import shutil

import pytest

from oracle import variants as V
from tests import test_oracle_var_pins as P

SRC = os.path.join(os.path.dirname(V.__file__), "efunc_oracle_var.c")
HDR = os.path.join(os.path.dirname(V.__file__), "efunc_oracle_var.h")

MUTANTS = {
    "quadratic_half_dropped": ("mono[4] = 0.5 * x[0] * x[0];", "mono[4] = x[0] * x[0];"),
    "cross_term_wrong_axis": ("mono[8] = x[0] * x[2];", "mono[8] = x[1] * x[2];"),
    "value_grad_missing_diagonal": ("g[0] += sxx * x[0] + sxy * x[1] + sxz * x[2];",
                                    "g[0] += sxy * x[1] + sxz * x[2];"),
    "value_grad_transposed": ("g[1] += sxy * x[0] + syy * x[1] + syz * x[2];",
                              "g[1] += sxz * x[0] + syy * x[1] + syz * x[2];"),
    "beta_grad_sign": ("t[3] = dl * (-x2n) * r;", "t[3] = dl * (x2n) * r;"),
    "centre_grad_factor_2": ("t[d] = dl * (-df[d] + 2.0 * k[3] * x[d] * r);",
                             "t[d] = dl * (-df[d] + k[3] * x[d] * r);"),
    "rho_chain_rule_missing": ("if (m->learn_scale) t[ro] = exp((double)p[ro]) * gg[3];",
                               "if (m->learn_scale) t[ro] = gg[3];"),
    "offset_sign": ("for (int d = 0; d < 3; ++d) k[d] += (double)p[L[2] + d];",
                    "for (int d = 0; d < 3; ++d) k[d] -= (double)p[L[2] + d];"),
    "fixed_scale_ignored": ("k[3] = m->learn_scale ? exp((double)p[ro]) : exp(m->rho_fixed);",
                            "k[3] = m->learn_scale ? exp((double)p[ro]) : 1.0;"),
    "scale_before_values": ("        l[0] = c; c += nv;\n        if (m->learn_scale) { l[1] = c; c += 1; }",
                            "        if (m->learn_scale) { l[1] = c; c += 1; }\n        l[0] = c; c += nv;"),
    # the tolerance scales the variant parity checks rest on
    "sigma_not_normalised": ("*sigma = sa / e;", "*sigma = sa;"),
    "kappa_x100": ("kk += wr * fabs(s);", "kk += 100.0 * wr * fabs(s);"),
    "tail_x10": ("if (s - lse < -T) tl += wr;", "if (s - lse < -T) tl += 10.0 * wr;"),
    "grad_scale_x10": ("adl = fabs(dLdO[j]) * w;", "adl = 10.0 * fabs(dLdO[j]) * w;"),
    "grad_scale_signed_monomial": ("ta[4 + c] = adl * fabs(mono[c]);", "ta[4 + c] = adl * mono[c];"),
    "subthreshold_wrong_side": ("const int below = lw < -T;", "const int below = lw > -T;"),
    "qsig_drops_curvature": ("g[0] += fabs(sxx * x[0]) + fabs(sxy * x[1]) + fabs(sxz * x[2]);",
                             "g[0] += fabs(sxy * x[1]) + fabs(sxz * x[2]);"),
    "qkap_x100": ("qk[d] += w * fabs(s) * fabs(ga - G[d])", "qk[d] += 100.0 * w * fabs(s) * fabs(ga - G[d])"),
    "qtail_drops_renormalisation": ("if (below) qt[d] += w * (fabs(ga) + fabs(G[d]));",
                                    "if (below) qt[d] += w * fabs(ga);"),
}

PINS = [getattr(P, n) for n in dir(P) if n.startswith("test_")]


def _run_pins(var):
    for fn in PINS:
        kwargs_list = [{}]
        for mk in getattr(fn, "pytestmark", []):
            if mk.name == "parametrize":
                name, vals = mk.args
                kwargs_list = [{name: v} for v in vals]
        for kw in kwargs_list:
            try:
                fn(var, **kw)
            except AssertionError:
                return fn.__name__
            except Exception:  # noqa: BLE001 - a crash also counts as caught
                return fn.__name__ + " (error)"
    return None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_var_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {name}"
    shutil.copy(HDR, tmp_path / "efunc_oracle_var.h")
    (tmp_path / "efunc_oracle_var.c").write_text(src.replace(old, new))
    lib = V.build_var_oracle(force=True, src=str(tmp_path / "efunc_oracle_var.c"),
                             out=str(tmp_path / "libmutant.so"))
    V.load()
    prev = V.use_library(lib)
    try:
        caught = _run_pins(V)
    finally:
        V.restore(prev)
    assert caught, f"no pin caught mutant {name}"
