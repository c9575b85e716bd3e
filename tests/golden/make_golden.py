"""Writes tests/golden/oracle_ipm.json: the FP64 oracle's interior-point results
on the seeded workloads (iterations, objective, final residuals, mu trace).

Calls only the oracle and the instance generator.  Run from the repository
root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bounded  # noqa: E402
from oracle import general as ogeneral  # noqa: E402
from oracle import ipm  # noqa: E402
from paper_2412_07731_amd import gen  # noqa: E402


def traces(r):
    """Per-iteration records of an oracle run and its start solves."""
    return dict(mu_trace=[h["mu"] for h in r.history],
                sigma_trace=[h["sigma"] for h in r.history],
                alpha_p=[h["ap"] for h in r.history],
                alpha_d=[h["ad"] for h in r.history],
                # backward errors after refinement of the predictor and the
                # corrector of every iteration, and of the two start solves
                bkerr_pred=[h["bkerr_pred"] for h in r.history],
                bkerr_corr=[h["bkerr"] for h in r.history],
                start_bkerr=[r.solves[0][0], r.solves[1][0]],
                correctors=sum(h.get("correctors", 0) for h in r.history),
                correctors_trace=[h.get("correctors", 0) for h in r.history],
                # refinement corrections of every solve in call order (the two
                # start solves, then each iteration's predictor, corrector and
                # any correctors)
                refine_trace=[steps for _, steps in r.solves])


def run_general(config, seed, dense=False, x0_border=False, bounds=False):
    """General-form instance (bounds, inequality rows): the oracle's
    reformulation and IPM; objective in the general form's variables.  With
    dense, the global rows stay whole in the border of the Schur complement
    (the dense layer; with x0_border the x_0-only equality rows too), and the
    trajectory is recorded."""
    g = gen.generate_general(config, seed)
    t = time.time()
    x, f, r = ogeneral.solve(g, dense=dense, x0_border=x0_border, bounds=bounds)
    out = dict(config=config, seed=seed, gondzio=0, status=r.status, iterations=r.iterations,
               objective=f, pobj_std=r.pobj, relgap=r.relgap, pinf=r.pinf, dinf=r.dinf,
               mu=r.mu, seconds=round(time.time() - t, 2))
    if dense or bounds:
        out.update(**traces(r))
    if dense:
        out["dense"] = True
        if x0_border:
            out["x0_border"] = True
    if bounds:
        out["bounds"] = True
    return out


def run(config, seed, gondzio=0, dense=False, x0_border=False, bounds=False):
    if config in gen.GENERAL_CONFIGS:
        return run_general(config, seed, dense, x0_border, bounds)
    inst = gen.generate(config, seed)
    t = time.time()
    if getattr(inst, "ub", None) is not None:     # upper bounds inside the iteration
        r = bounded.solve(inst, ipm.Options(gondzio=gondzio))
    else:
        r = ipm.solve(inst, ipm.Options(gondzio=gondzio))
    return dict(config=config, seed=seed, gondzio=gondzio, status=r.status, iterations=r.iterations,
                pobj=r.pobj, dobj=r.dobj, relgap=r.relgap, pinf=r.pinf, dinf=r.dinf,
                mu=r.mu, fstar=inst.fstar, refine_steps=r.refine_steps,
                max_bkerr=r.max_bkerr, pivots=r.pivots, **traces(r),
                seconds=round(time.time() - t, 2))


def main():
    """No arguments: rewrite the file with tiny (seeds 0-7) and n512 (seed 0).
    --quick: tiny only.  --refresh: run again every run the file holds.
    --add CONFIG:SEED[:gK][:dense|:dense_x0][:bounds] [...]: run just those
    (with K Gondzio correctors per iteration if gK is given; a general-form
    instance through the dense layer with :dense, with its x_0-only rows in the
    border too with :dense_x0, with its upper bounds inside the iteration with
    :bounds) and merge them into the existing file (e.g.
    --add uneven:0, the N=2048 workload, which takes minutes and several GB;
    --add g_medium:0, a general-form instance; --add tiny_g:0, global rows)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_ipm.json")
    if "--add" in sys.argv or "--refresh" in sys.argv:
        out = json.load(open(path))
        if "--refresh" in sys.argv:
            specs = [f"{q['config']}:{q['seed']}" + (f":g{q['gondzio']}" if q.get("gondzio") else "")
                     + (":dense_x0" if q.get("x0_border") else ":dense" if q.get("dense") else "")
                     + (":bounds" if q.get("bounds") else "")
                     for q in out["runs"]]
        else:
            specs = sys.argv[sys.argv.index("--add") + 1:]
        for spec in specs:
            parts = spec.split(":")
            config, seed = parts[0], int(parts[1])
            x0b = "dense_x0" in parts[2:]
            dense = x0b or "dense" in parts[2:]
            bnds = "bounds" in parts[2:]
            gk = [q for q in parts[2:] if q.startswith("g")]
            g = int(gk[0][1:]) if gk else 0      # CONFIG:SEED:gK = K correctors
            r = run(config, seed, g, dense, x0b, bnds)
            key = (config, seed, g, dense, x0b, bnds)
            out["runs"] = [q for q in out["runs"]
                           if (q["config"], q["seed"], q.get("gondzio", 0), q.get("dense", False),
                               q.get("x0_border", False), q.get("bounds", False)) != key]
            out["runs"].append(r)
            print(config, seed, g, parts[2:], r["status"], r["iterations"], r["seconds"], "s",
                  flush=True)
    else:
        out = {"note": "FP64 oracle results; written by tests/golden/make_golden.py",
               "runs": []}
        for seed in range(8):
            out["runs"].append(run("tiny", seed))
        if "--quick" not in sys.argv:
            out["runs"].append(run("n512", 0))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
