"""The count and margin pins catch plausible slips in the oracle.

Each case copies oracle/lf_oracle.c, plants one mistake of the kind that
would go unnoticed by the radiance and gradient pins (a strict instead of a
non-strict bound, a count of the wrong crossings, a margin measured against
the wrong switching point), builds the copy into a temporary library, binds
it in place of the oracle and runs every pin of tests/test_oracle_counts.py:
at least one must fail.  The oracle itself is never modified.  CPU only."""
import concurrent.futures as cf
import os

import pytest

import oracle
from oracle import build as obuild
from tests import test_oracle_counts as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lf_oracle.c")

MUTANTS = {
    # crossings at t = t_(k) no longer touched
    "touch_strict_at_kth": ("c->t > p->t_min && c->t <= tk) st->touch += 1.0;",
                            "c->t > p->t_min && c->t < tk) st->touch += 1.0;"),
    # crossings below the opacity threshold counted twice
    "touch_faint_twice": ("st->touch += 1.0;", "st->touch += c->valid ? 1.0 : 2.0;"),
    # only valid hits counted as touched
    "touch_valid_only": ("if (c->in3s && c->t > p->t_min", "if (c->valid && c->t > p->t_min"),
    # t_(k) taken as the (k+1)-th hit
    "kth_off_by_one": ("double tk = nv >= k ? buf->c[k - 1].t : INFINITY;",
                       "double tk = nv > k ? buf->c[k].t : INFINITY;"),
    # the t gap taken over the first k hits instead of k+1
    "tgap_over_k": ("int64_t lim = nv < k + 1 ? nv : k + 1;", "int64_t lim = nv < k ? nv : k;"),
    # the support margin against the 3-sigma radius instead of the combined bound
    "rho_margin_vs_sigma": ("st->rho = dmin(st->rho, fabs(c->rho2 - c->rho2max));",
                            "st->rho = dmin(st->rho, fabs(c->rho2 - sig2));"),
    # the t_min margin measured from zero
    "tmin_margin_from_zero": ("st->tmin = dmin(st->tmin, fabs(c->t - p->t_min));",
                              "st->tmin = dmin(st->tmin, fabs(c->t));"),
    # composited secondary hits counted once per ray
    "comp2_per_ray": ("fz->counts[ORS_C_COMP_SEC] += hl2->nh;", "fz->counts[ORS_C_COMP_SEC] += 1.0;"),
    # the secondary trace's statistics merged into the primary's
    "sec_stats_into_primary": ("trace_decide(w, o2, sp->w, p->k, buf, hl2, &st2);",
                               "trace_decide(w, o2, sp->w, p->k, buf, hl2, &st);"),
    # the E(w) lookup counted only for traced samples
    "env_count_after_trace": ("    sp->live = 1;\n    fz->counts[ORS_C_ENV] += 1.0;\n",
                              "    sp->live = 1;\n    if (!(p->flags & ORS_NO_SECONDARY)) fz->counts[ORS_C_ENV] += 1.0;\n"),
    # the row-CDF margin measured with the column uniform
    "env_margin_wrong_uniform": ("fabs(w->cdf_row[r + 1] - ua));", "fabs(w->cdf_row[r + 1] - ub));"),
    # the lobe margin against a fixed one half
    "lobe_margin_vs_half": ("fz->margins[ORS_M_LOBE] = dmin(fz->margins[ORS_M_LOBE], fabs(u1 - qs));",
                            "fz->margins[ORS_M_LOBE] = dmin(fz->margins[ORS_M_LOBE], fabs(u1 - 0.5));"),
    # the hemisphere margin from the world up axis instead of the normal
    "cos_margin_world_axis": ("fz->margins[ORS_M_COS] = dmin(fz->margins[ORS_M_COS], fabs(cosw));",
                              "fz->margins[ORS_M_COS] = dmin(fz->margins[ORS_M_COS], fabs(sp->w[2]));"),
}


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    src = open(SRC).read()
    d = tmp_path_factory.mktemp("mutants")
    jobs = {}
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, f"{name}: the planted line must occur exactly once"
        path = d / f"{name}.c"
        path.write_text(src.replace(old, new))
        jobs[name] = (str(path), str(d / f"lib{name}.so"))
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {n: ex.submit(obuild.build, False, s, o) for n, (s, o) in jobs.items()}
        return {n: f.result() for n, f in futs.items()}


def _failures():
    failed = []
    for fn, cases in pins.PINS:
        for args in cases:
            try:
                fn(*args)
            except AssertionError:
                failed.append(f"{fn.__name__}{args}")
    return failed


def test_pins_pass_on_the_oracle():
    assert _failures() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_slip_fails_a_pin(mutant_libs, monkeypatch, name):
    monkeypatch.setattr(oracle, "_lib", oracle.bind(mutant_libs[name]))
    assert _failures(), f"no pin caught the planted slip {name}"
