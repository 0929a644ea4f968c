"""Write tests/golden/oracle_small.json from the FP64 oracle only.

The paper prints no worked numeric example for the dense objective, so the stored
values are a regression snapshot of the oracle (already pinned by
tests/test_oracle_pins.py) on a small seeded case: eq. 1 (D), eq. 5 (S), eq. 9
(Vhat), eq. 10 (K), eq. 11 (J) at u = 0 and u = u_true, the adaptive keypoint
weight of Sec. II-D2, and gradient / GN-product norms.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def snapshot():
    d = synth.small_pair(shape=(16, 16, 12), spacing=(1.5, 1.5, 1.5), seed=3)
    P = oracle.Problem(d["R"], d["T"], d["spacing"], d["kp_x"], d["kp_t"],
                       oracle.Weights(eta=10.0, alpha=1.0, gamma=0.1))
    u0 = np.zeros(d["u_true"].shape)
    P.w.delta = P.adaptive_delta(u0)
    out = {"case": "synth.small_pair(shape=(16,16,12), spacing=(1.5,1.5,1.5), seed=3); "
                   "eta=10, alpha=1, gamma=0.1, delta adaptive at u=0",
           "delta": P.w.delta}
    for name, u in (("u0", u0), ("u_true", d["u_true"].astype(np.float64))):
        lin = P.linearise(u)
        hv = P.gn_hv(d["v"].astype(np.float64))
        out[name] = {k: float(lin[k]) for k in ("J", "D", "S", "V", "K")}
        out[name]["grad_l2"] = float(np.linalg.norm(lin["g"]))
        out[name]["diag_l2"] = float(np.linalg.norm(lin["diag"]))
        out[name]["hv_l2"] = float(np.linalg.norm(hv))
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small.json")
    with open(path, "w") as f:
        json.dump(snapshot(), f, indent=1, sort_keys=True)
    print("wrote", path)
