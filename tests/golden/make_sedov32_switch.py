"""Write tests/golden/sedov32_switch_particle.json and sedov32_guard_particle.json.

Runs the oracle alone (no GPU code) on the point explosion of sec. 3.1.5 at
32^3 (workloads.sedov_point(32), MFM, gamma 5/3, N_NGB 32) towards t = 0.1 and
records, for the close of the step (sec. 2.3.7), the first particle that
meets each of two conditions, with its start-of-step state, its flux sum dQ
and the step dt:

* switch: the integrated internal energy exceeds alpha_1 E_kin while
  E - E_kin < 0, so that recovering U from the total energy whenever the
  integrated U exceeds alpha_1 E_kin would make it negative;
* guard: neither the integrated U nor E - E_kin is positive.

Usage: python tests/golden/make_sedov32_switch.py   (about five minutes)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2211_12243_amd import workloads as W  # noqa: E402

KEYS = ("x", "y", "z", "m", "vx", "vy", "vz", "E", "U")


def record(st, out, i, step, t, kind):
    rec = {k: float(st[k][i]) for k in KEYS}
    rec.update({"dQ": [float(v) for v in out["fluxes"]["dQ"][:, i]], "dt": float(out["dt"]),
                "step": step, "t": t, "particle": int(i), "kind": kind,
                "source": "oracle, workloads.sedov_point(32), MFM, to t = 0.1"})
    return rec


def main():
    st, _ = W.sedov_point(32)
    cfg = {"scheme": "mfm", "gamma": 5.0 / 3.0, "n_ngb": 32.0}
    alpha1 = 0.01
    t, step, t_end = 0.0, 0, 0.1
    found = {}
    while t < t_end * (1.0 - 1e-12) and len(found) < 2:
        out = oracle.pipeline(cfg, st, t_end - t)
        dQ = out["fluxes"]["dQ"]
        m = st["m"]
        v0 = np.stack([st["vx"], st["vy"], st["vz"]])
        p1 = m * v0 + dQ[1:4]
        ekin1 = (p1 * p1).sum(0) / (2.0 * m)
        u_int = st["U"] + dQ[4] - (v0 * dQ[1:4]).sum(0) + 0.5 * (v0 * v0).sum(0) * dQ[0]
        e_kin = st["E"] + dQ[4] - ekin1
        sw = np.where((u_int > alpha1 * ekin1) & (e_kin < 0.0))[0]
        gd = np.where((u_int <= 0.0) & (e_kin <= alpha1 * ekin1))[0]
        if sw.size and "switch" not in found:
            found["switch"] = record(st, out, sw[0], step, t, "switch")
        if gd.size and "guard" not in found:
            found["guard"] = record(st, out, gd[0], step, t, "guard")
        st = out["state"]
        t += out["dt"]
        step += 1
        print(step, f"t={t:.4e}", sorted(found), flush=True)
    for kind, rec in found.items():
        with open(os.path.join(HERE, f"sedov32_{kind}_particle.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    main()
