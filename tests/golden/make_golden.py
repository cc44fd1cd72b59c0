"""Write the stored expected values of the long-horizon parity tests.

Every value here comes from the FP64 oracle (``oracle/``) run on the seeded
inputs of ``paper_2112_02574_amd.inputs``; nothing is read from the GPU
library.  Usage (repository root):

    python tests/golden/make_golden.py c1      # 64^2 slab, 2000 steps
    python tests/golden/make_golden.py c2      # 4 x 256^2 droplets, 20000 steps
    python tests/golden/make_golden.py c2conv  # the same run to the Sec. 4 dP criterion
    python tests/golden/make_golden.py c3      # 128^3 droplet, 30000 steps

Each writes tests/golden/<name>_oracle.json.  The droplet cases start the way
Sec. 4 does: a flat interface with the same couplings is relaxed first (the
oracle's ``flat_equilibrium``) and the droplet's tanh profile then joins its
two bulk concentrations; the stored ``bulk`` values let a checked run start
from the identical fields.  ORACLE_THREADS sets the OpenMP threads.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2112_02574_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
G_SYM = ((0.0, 1.8), (1.8, 0.0))
THREADS = int(os.environ.get("ORACLE_THREADS", "0"))


def flat_bulk(dim, order, g, lx=128):
    """Stage one of the Sec. 4 initialisation, on the oracle."""
    t0 = time.time()
    bulk, steps = O.flat_equilibrium(dim, order, g, lx=lx, guess=inputs.FLAT_GUESS[g[0][0]],
                                     tol=1e-10, nthreads=1)
    print(f"flat stage d={dim} E{order}: {bulk} after {steps} steps ({time.time() - t0:.0f} s)",
          flush=True)
    return bulk, steps


def _write(name, payload):
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as fh:
        json.dump(payload, fh, indent=1)
        fh.write("\n")
    print("wrote", path, flush=True)


def c1():
    """D2Q9, E4, 64x64, tau = 1, g_AB = 1.8, psi = n; slab with noise 1e-3
    (splitmix64 seed 1); 2000 steps.  y-averaged profiles and sigma0."""
    o = O.Oracle(2, 4, (64, 64), tau=1.0, g=G_SYM)
    o.set_density(*inputs.slab(64, 64, noise=1e-3, seed=1))
    o.run(2000)
    n = o.density()[:, 0]
    s0, PN, PT = o.flat_sigma0()
    st = o.stats()
    _write("c1", {"steps": 2000, "nA_profile": n[0].mean(axis=0).tolist(),
                  "nB_profile": n[1].mean(axis=0).tolist(),
                  "nA_field_row0": n[0][0].tolist(), "sigma0": s0,
                  "PN": PN.tolist(), "PT": PT.tolist(), "mass": st["mass"].tolist(),
                  "max_u": st["max_u"]})


def c2():
    """D2Q9, E8, 256x256, four A-rich droplets R0 in {12, 20, 32, 48};
    20000 steps.  Droplet observables (2D forms)."""
    bulk, fsteps = flat_bulk(2, 8, G_SYM)
    out = {"steps": 20000, "bulk": bulk, "flat_steps": fsteps, "flat_lx": 128, "members": []}
    for R0 in (12.0, 20.0, 32.0, 48.0):
        t0 = time.time()
        o = O.Oracle(2, 8, (256, 256), tau=1.0, g=G_SYM, nthreads=THREADS)
        o.set_density(*inputs.droplet(256, 256, R=R0, bulk=bulk))
        o.run(20000)
        d = o.droplet_observables(R0)
        d = {k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in d.items()}
        d["R0"] = R0
        d["max_u"] = o.stats()["max_u"]
        out["members"].append(d)
        print(f"c2 R0={R0}: dP={d['dP']:.6g} R_s={d['R_s']:.6g} ({time.time() - t0:.0f} s)",
              flush=True)
    _write("c2", out)


def c2conv(every=2048, tol=1e-5, max_steps=400000):
    """The four droplets of c2 run on until the Delta P criterion of Sec. 4:
    |dP(t) - dP(t - 2^11)| / |dP(t - 2^11)| < 1e-5.  Per member: the step at
    which it holds, the observables there and the dP, R_s history."""
    bulk, fsteps = flat_bulk(2, 8, G_SYM)
    out = {"every": every, "tol": tol, "bulk": bulk, "flat_steps": fsteps, "flat_lx": 128,
           "members": []}
    for R0 in (12.0, 20.0, 32.0, 48.0):
        t0 = time.time()
        o = O.Oracle(2, 8, (256, 256), tau=1.0, g=G_SYM, nthreads=THREADS)
        o.set_density(*inputs.droplet(256, 256, R=R0, bulk=bulk))
        hist, done, prev = [], 0, None
        while done < max_steps:
            o.run(every)
            done += every
            d = o.droplet_observables(R0)
            hist.append({"step": done, "dP": d["dP"], "R_s": d["R_s"]})
            change = abs(d["dP"] - prev) / abs(prev) if prev else float("inf")
            prev = d["dP"]
            if change < tol:
                break
        d = {k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in d.items()}
        d.update({"R0": R0, "steps": done, "converged": change < tol, "history": hist,
                  "max_u": o.stats()["max_u"]})
        out["members"].append(d)
        print(f"c2conv R0={R0}: {done} steps, dP={d['dP']:.8g} R_s={d['R_s']:.8g} "
              f"({time.time() - t0:.0f} s)", flush=True)
    _write("c2conv", out)


def c3(steps=30000, every=2048):
    """D3Q19, E6, 128^3 droplet R0 = 24, tau = 1, g_AB = 1.8; observables every
    2048 steps (the paper's monitoring interval) and at the end."""
    L, R0 = 128, 24.0
    bulk, fsteps = flat_bulk(3, 6, G_SYM)
    o = O.Oracle(3, 6, (L, L, L), tau=1.0, g=G_SYM, nthreads=THREADS)
    o.set_density(*inputs.droplet(L, L, L, R=R0, bulk=bulk))
    hist = []
    done = 0
    t0 = time.time()
    while done < steps:
        k = min(every, steps - done)
        o.run(k)
        done += k
        d = o.droplet_observables(R0)
        st = o.stats()
        hist.append({"step": done, "dP": d["dP"], "R_s": d["R_s"], "sigma_s": d["sigma_s"],
                     "C_d": d["C_d"], "max_u": st["max_u"], "mass": st["mass"].tolist()})
        print(f"c3 step {done}: dP={d['dP']:.6g} R_s={d['R_s']:.6g} "
              f"max_u={st['max_u']:.3g} ({time.time() - t0:.0f} s)", flush=True)
    d = o.droplet_observables(R0)
    final = {k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in d.items()}
    n = o.density()
    final["nA_axis"] = n[0, L // 2, L // 2, :].tolist()
    final["nB_axis"] = n[1, L // 2, L // 2, :].tolist()
    _write("c3", {"steps": steps, "bulk": bulk, "flat_steps": fsteps, "flat_lx": 128,
                  "history": hist, "final": final})


if __name__ == "__main__":
    {"c1": c1, "c2": c2, "c2conv": c2conv, "c3": c3}[sys.argv[1]]()
