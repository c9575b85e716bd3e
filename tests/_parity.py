"""Shared checks of the GPU parity tests against the oracle's recorded runs
(tests/golden/oracle_ipm.json).  Not a test module."""
import json
import os

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_ipm.json")))

# Backward-error target of a Newton direction (relative KKT residual on the
# unregularized Newton system of Sec. 2.3).  Along an interior-point run the
# oracle itself misses it in the last iterations, where the system is nearly
# singular, so an iterate passes if its direction is within 10x of the
# oracle's backward error on the same iterate.
ETA = 1e-10


def golden(config, seed, gondzio=0, dense=False, x0_border=False, bounds=False):
    for r in GOLDEN["runs"]:
        if (r["config"] == config and r["seed"] == seed and r.get("gondzio", 0) == gondzio
                and r.get("dense", False) == dense and r.get("x0_border", False) == x0_border
                and r.get("bounds", False) == bounds):
            return r
    return None


# Refinement corrections per solve (the interior-point default of both sides).
MAX_REFINE = 5


def eta_bound(eta_orc, budget_limited=False):
    """Bound on the GPU's backward error for a solve where the oracle reached
    eta_orc.  Where the oracle used its whole refinement budget and still
    missed 1e-10 (a slowly contracting refinement late in a run), the final
    backward error is set by that budget, and the two sides' can differ by
    more: there the bound is 100 eta_orc."""
    return max(ETA, (100.0 if budget_limited else 10.0) * eta_orc)


def check_trajectory(hist, res, g, label, mu_rtol_early=1e-6, mu_rtol_late=1e-5, late=3):
    """Per-iterate parity of an FP64 interior-point run with the oracle's run
    of the same instance: the same number of iterations; for every predictor
    and corrector (and the two start-point solves) a backward error after
    refinement of at most max(1e-10, 10 eta_orc) (100 eta_orc where the
    oracle's refinement ran out of corrections, see eta_bound); mu at the top of every
    iteration within mu_rtol_early of the oracle's (mu_rtol_late in the last
    `late` iterations, where the directions are ill-conditioned and rounding
    differences grow).  Where the oracle's run records its refinement counts
    (refine_trace), mu is compared only up to the first iteration in which one
    side refined a direction and the other did not (both met the acceptance
    test, from either side of it; from there the two runs follow different,
    equally valid directions); the backward errors are still checked at every
    iterate.  Returns (iterates missing 1e-10 itself, worst mu relative
    difference)."""
    assert len(hist) == g["iterations"], (label, len(hist), g["iterations"])
    misses = 0
    rt = g.get("refine_trace") if not g.get("correctors") else None

    def capped(idx, eo):     # the oracle's solve idx used its whole budget and missed 1e-10
        return rt is not None and rt[idx] >= MAX_REFINE and eo > ETA

    for j, (eg, eo) in enumerate(zip(res["start_bkerr"], g["start_bkerr"])):
        assert eg <= eta_bound(eo, capped(j, eo)), (label, "start", j, eg, eo)
        misses += eg > ETA
    worst_mu = 0.0
    n = len(hist)
    branch = None
    for k, h in enumerate(hist):
        for q, key in enumerate(("bkerr_pred", "bkerr_corr")):
            eg, eo = h[key], g[key][k]
            assert eg <= eta_bound(eo, capped(2 + 2 * k + q, eo)), (label, k, key, eg, eo)
            misses += eg > ETA
        if branch is None:
            mo = g["mu_trace"][k]
            d = abs(h["mu"] - mo) / mo
            worst_mu = max(worst_mu, d)
            tol = mu_rtol_late if k >= n - late else mu_rtol_early
            assert d <= tol, (label, k, "mu", h["mu"], mo)
        if rt is not None and branch is None:
            if ((h["refine_pred"] > 0) != (rt[2 + 2 * k] > 0)
                    or (h["refine_corr"] > 0) != (rt[3 + 2 * k] > 0)):
                branch = k
    note = "" if branch is None else f"; refinement decisions part at iteration {branch}"
    print(f"{label}: {n} iterations, {misses} of {2 * n + 2} solves above eta = {ETA:g} "
          f"(oracle: {sum(e > ETA for e in g['bkerr_pred'] + g['bkerr_corr'] + g['start_bkerr'])}), "
          f"worst mu difference {worst_mu:.1e}{note}", flush=True)
    return misses, worst_mu
