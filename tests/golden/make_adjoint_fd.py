"""Write ``adjoint_fd.json``: interface-height losses of the FP64 oracle and their
central finite differences, the reference of the reverse-mode tests.

Calls only the oracle (through ``tests/_adjoint_ref.py``) and the seeded
input generators of ``paper_2207_14496_amd.setups``.  Run from the repository
root:  python tests/golden/make_adjoint_fd.py  (about ten minutes on 8 cores).

Workload: the 2-D standing wave of Sec. 4.1 (FP64, SRT, EQ refilling, sigma = 0)
at two sizes.  One size has 64 x 128 cells, depth 64 and a0 = 0.64.  The other
has 128 x 256 cells, depth 128 and a0 = 1.28, and is the differentiable
configuration.  A third, calm wave (64 x 128, depth 64.5, a0 = 0.3) keeps its
surface inside one row of interface cells for 1500 steps: no cell converts,
and over that many steps viscous damping makes dL/domega large enough to
resolve.  Loss L = mean over t = 1..T of (h(t) - h*(t))^2, with h(t) the
summed fill level on the plane x = 32.  The target h* comes from an oracle run
at omega (1 + xi1), g (1 + xi2), a0 (1 + xi3), with the xi drawn per seed by
``setups.target_perturbation``.

Reference derivative: the four-point central difference
    (8 (L(p+d) - L(p-d)) - (L(p+2d) - L(p-2d))) / (12 d).
The step d is the largest on a ladder whose four runs, and those of the next
smaller step (kept as a confirmation), reproduce the unperturbed cell-type
sequence.  Near that step, FP64 rounding of the trajectory (about 1e-14 in L)
limits plain two-point differences at d = 1e-6 p to about 1e-5 relative for
omega and g.
"""
from __future__ import annotations

import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import _adjoint_ref as R  # noqa: E402
from paper_2207_14496_amd import setups  # noqa: E402

PARAM_LADDER = (1e-3, 3e-4, 1e-4, 3e-5, 1e-5)     # relative steps
STATE_LADDER = (1e-3, 3e-4, 1e-4, 3e-5, 1e-5)     # absolute steps
X_PROBE = 32

W64 = dict(nx=64, ny=128, depth=64.0, a0=0.64, omega=1.8, g=1e-5)
W128 = dict(nx=128, ny=256, depth=128.0, a0=1.28, omega=1.8, g=1e-5)
# a calm wave: the surface stays inside one row of interface cells, so no cell
# converts over a window long enough for viscous damping to make dL/domega
# resolvable to well below 1e-6 by differences with large steps
W64C = dict(nx=64, ny=128, depth=64.5, a0=0.3, omega=1.8, g=1e-5)

CASES = [
    # conversion-free windows (the first conversion comes at step 64 in both)
    dict(name="wave64_T60", geo=W64, T=60, seeds=[0, 1], cells=True),
    dict(name="wave128_T60", geo=W128, T=60, seeds=[0, 1], cells=True),
    # windows with conversions; per-domain base parameters differ
    dict(name="wave64_T300", geo=W64, T=300, seeds=[0, 1, 2], cells=True, vary=True),
    # the differentiable configuration over a window with conversions (over the
    # full 4000 steps, about 3100 conversions per domain, and already over 400
    # steps, no step of the ladder keeps the cell-type sequence for g and a0)
    dict(name="wave128_T200", geo=W128, T=200, seeds=[0, 7], cells=False,
         ladder=(1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6)),
    # conversion-free over 1500 steps: all three derivatives to 1e-6, omega included
    dict(name="wave64_calm_T1500", geo=W64C, T=1500, seeds=[1, 2, 3], cells=False,
         ladder=(1e-2, 3e-3, 1e-3, 3e-4)),
]


def base_params(case, seed):
    g = case["geo"]
    p = dict(omega=g["omega"], g=g["g"], a0=g["a0"])
    if case.get("vary"):
        p = dict(omega=g["omega"] + 0.02 * seed, g=g["g"] * (1.0 + 0.1 * seed),
                 a0=g["a0"] * (1.0 + 0.05 * seed))
    return p


def _run(job):
    """One oracle loss run.  job = (geo, params, target, T, state_edit)."""
    geo, prm, target, T, edit = job
    p, st = R.wave_state(geo["nx"], geo["ny"], geo["depth"], prm["a0"], prm["omega"], prm["g"])
    if edit is not None:
        field, idx, delta = edit
        arr = {"phi": st.phi, "m": st.m, "f": st.f}[field]
        arr[tuple(idx) if isinstance(idx, list) else idx] += delta
    L, h, dig, nconv = R.run_loss(p, st, target, T, X_PROBE)
    return L, dig, st.flags.tobytes(), nconv, h


def _target(job):
    geo, prm, seed, T = job
    return R.seeded_target(geo["nx"], geo["ny"], geo["depth"], prm["a0"], prm["omega"], prm["g"], seed,
                           T, X_PROBE).tolist()


def pick_cells(geo, prm):
    """Interface cells on and next to the probe plane, and PDF entries of an
    interface and a liquid cell under the probe."""
    p, st = R.wave_state(geo["nx"], geo["ny"], geo["depth"], prm["a0"], prm["omega"], prm["g"])
    nx = geo["nx"]
    fl = st.flags.reshape(geo["ny"], nx)
    out = []
    for x in (X_PROBE, X_PROBE - 1, X_PROBE + 3):
        ys = np.nonzero(fl[:, x] == 2)[0]
        cell = int(ys[len(ys) // 2] * nx + x)
        out.append(("phi", cell))
        out.append(("m", cell))
    ys = np.nonzero(fl[:, X_PROBE] == 2)[0]
    cif = int(ys[0] * nx + X_PROBE)
    cliq = int((ys[0] - 2) * nx + X_PROBE)
    for i in (0, 3, 4, 8):
        out.append(("f", [i, cif]))
        out.append(("f", [i, cliq]))
    return out


def c4(v, d):
    return (8.0 * (v[1] - v[-1]) - (v[2] - v[-2])) / (12.0 * d)


def main(only=None):
    procs = min(8, os.cpu_count() or 1)
    path = os.path.join(HERE, "adjoint_fd.json")
    out = {"x_probe": X_PROBE, "param_ladder": PARAM_LADDER, "state_ladder": STATE_LADDER, "cases": []}
    if only and os.path.exists(path):
        with open(path) as fh:
            out = json.load(fh)
        out["cases"] = [c for c in out["cases"] if c["name"] not in only and
                        c["name"] in {k["name"] for k in CASES}]
    with Pool(procs) as pool:
        for case in CASES:
            if only and case["name"] not in only:
                continue
            geo, T = case["geo"], case["T"]
            seeds = case["seeds"]
            prms = [base_params(case, s) for s in seeds]
            targets = pool.map(_target, [(geo, prm, s, T) for prm, s in zip(prms, seeds)])
            jobs, keys = [], []
            cells = {}
            for si, (s, prm) in enumerate(zip(seeds, prms)):
                jobs.append((geo, prm, targets[si], T, None))
                keys.append((si, "base", None, None, 0))
                for name in ("omega", "g", "a0"):
                    for rel in case.get("ladder", PARAM_LADDER):
                        d = rel * abs(prm[name])
                        for k in (-2, -1, 1, 2):
                            q = dict(prm)
                            q[name] = prm[name] + k * d
                            jobs.append((geo, q, targets[si], T, None))
                            keys.append((si, "param", name, rel, k))
                if case.get("cells"):
                    cells[si] = pick_cells(geo, prm)
                    for ci, (field, idx) in enumerate(cells[si]):
                        for step in STATE_LADDER:
                            for k in (-2, -1, 1, 2):
                                jobs.append((geo, prm, targets[si], T, (field, idx, k * step)))
                                keys.append((si, "cell", ci, step, k))
            print(f"{case['name']}: {len(jobs)} oracle runs", flush=True)
            res = pool.map(_run, jobs, chunksize=1)
            table = dict(zip(keys, res))
            entries = []
            for si, (s, prm) in enumerate(zip(seeds, prms)):
                L0, dig0, fl0, nconv, h0 = table[(si, "base", None, None, 0)]

                def ladder(kind, key, steps, scale):
                    ok = []
                    for st in steps:
                        runs = [table[(si, kind, key, st, k)] for k in (-2, -1, 1, 2)]
                        same = all(r[1] == dig0 and r[2] == fl0 for r in runs)
                        ok.append((same, st, {k: r[0] for k, r in zip((-2, -1, 1, 2), runs)}))
                    for j in range(len(ok) - 1):
                        if ok[j][0] and ok[j + 1][0]:
                            d0, d1 = ok[j][1] * scale, ok[j + 1][1] * scale
                            return dict(ref=c4(ok[j][2], d0), confirm=c4(ok[j + 1][2], d1), step=ok[j][1])
                    return None

                grads = {n: ladder("param", n, case.get("ladder", PARAM_LADDER), abs(prm[n]))
                         for n in ("omega", "g", "a0")}
                ent = dict(seed=s, params=prm, xi=list(setups.target_perturbation(s)),
                           target=targets[si], loss=L0, conversions=nconv, grads=grads)
                if T <= 300:
                    ent["height"] = h0.tolist()
                if case.get("cells"):
                    ent["cells"] = []
                    for ci, (field, idx) in enumerate(cells[si]):
                        r = ladder("cell", ci, STATE_LADDER, 1.0)
                        ent["cells"].append(dict(field=field, index=idx, fd=r))
                entries.append(ent)
                print(f"  seed {s}: L={L0:.6e} conversions={nconv} grads=" +
                      str({k: (v['ref'] if v else None) for k, v in grads.items()}), flush=True)
            out["cases"].append(dict(name=case["name"], geometry=geo, T=T, entries=entries))
    order = [c["name"] for c in CASES]
    out["cases"].sort(key=lambda c: order.index(c["name"]))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote adjoint_fd.json")


if __name__ == "__main__":
    # optional arguments: case names to (re)compute; the others are kept
    main(sys.argv[1:] or None)
