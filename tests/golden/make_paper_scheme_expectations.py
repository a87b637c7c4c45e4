"""Writes paper_scheme_expectations.json: what the closed-form law of the
paper's election/selection scheme (oracle.laws.paper_law) predicts for the
Table 1 workloads -- the discrete Gaussian propensities of section "Test and
validation of the algorithm" with M = 64, 256, 1024 -- at thresholds
T_w = w * alpha_max, w in {1, 2}: the probability that an election fails
(no reaction eligible: the paper's rejection), and the expected MSE between
alpha / alpha_0 and the observed frequencies of n = 10^7 selections (the
frequencies normalised over the accepted selections):

    q = law / (1 - reject),  E[MSE] = mean_j (q_j - p_j)^2 + sum_j q_j (1 - q_j) / (n' M),
    n' = n (1 - reject).

Only the oracle is called.  Run from the repository root:
    python tests/golden/make_paper_scheme_expectations.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import laws  # noqa: E402
from paper_1404_0027_amd import workloads  # noqa: E402

N_SEL = 10_000_000


def main() -> None:
    out = {"source": "oracle.laws.paper_law on workloads.gaussian_vector(M)",
           "selections": N_SEL, "rows": {}}
    for M in (64, 256, 1024):
        a = workloads.gaussian_vector(M).astype(np.float64)
        p = a / a.sum()
        row = {}
        for w in (1, 2):
            law, rej = laws.paper_law(a, float(w))
            q = law / (1.0 - rej)
            n_acc = N_SEL * (1.0 - rej)
            mse = float(np.mean((q - p) ** 2) + np.sum(q * (1 - q)) / (n_acc * M))
            row[f"T{w}"] = {"reject_probability": float(rej),
                            "expected_rejections": float(N_SEL * rej),
                            "expected_mse": mse}
        row["exact_sampling_floor_mse"] = float(np.sum(p * (1 - p)) / (N_SEL * M))
        out["rows"][str(M)] = row
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "paper_scheme_expectations.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
