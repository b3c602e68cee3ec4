"""Writes c3_quadratic_forms.json: quadratic forms of the derivative workload
(N = 1e5, three d = 3 windows of N(0,1) features min-max scaled, l = (0.05,
0.1, 0.2), sigma_w = 1) computed by the FP64 direct-sum oracle only.

For V = workloads.derivative_c3_rhs(R = 8) and its first column alone (R = 1)
and each kernel (Gaussian, Matern-1/2, Matern-3/2):

  vKv      = sum_r v_r^T (sum_w sigma_w^2 K_w) v_r
  vdKdl[w] = sum_r v_r^T sigma_w^2 (dK_w/dl_w) v_r
  vdKds[w] = sum_r v_r^T 2 sigma_w K_w v_r

These are L = sum_r v_r^T K v_r and its gradients in l_w and sigma_w (the
backward of the quadratic loss), which need the full O(N^2) sums.
Usage: python tests/golden/make_c3_golden.py   (a few minutes on 8 cores)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402
from oracle.direct import oracle_direct  # noqa: E402

KERNELS = {"gaussian": WL.GAUSSIAN, "matern12": WL.MATERN12, "matern32": WL.MATERN32}


def forms(V, Y, dl, ds):
    return {"vKv": float(np.sum(V * Y)),
            "vdKdl": [float(np.sum(V * dl[w])) for w in range(dl.shape[0])],
            "vdKds": [float(np.sum(V * ds[w])) for w in range(ds.shape[0])]}


def main():
    V8 = WL.derivative_c3_rhs(R=8)
    out = {"workload": "derivative_c3(N=100000, seed=17343), V = derivative_c3_rhs(R=8, seed=17346)",
           "oracle": "oracle.direct.oracle_direct (FP64 direct sums)"}
    for name, k in KERNELS.items():
        p = WL.derivative_c3(N=100000, kernel=WL.GAUSSIAN)
        Y, dl, ds = oracle_direct(p.X, p.windows, k, p.ell, p.sigma, V8, want_derivs=True)
        out[name] = {"R1": forms(V8[:, :1], Y[:, :1], dl[:, :, :1], ds[:, :, :1]), "R8": forms(V8, Y, dl, ds)}
        print(name, out[name], flush=True)
    with open(os.path.join(HERE, "c3_quadratic_forms.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
