"""Write tests/golden/l3_exact.json: exact equilibrium averages of one L=3
Gaussian sample, by enumerating its 2^27 configurations.

Calls only the oracle package's brute-force enumerator (oracle/exact_enum.c)
and the seeded input generator.  Values: <H>/V, <(H/V)^2>, <q_l> and the
overlap distribution P(Q) (paper Sec. 2, Eqs. 1-4) at each temperature of an
8-point uniform grid on [0.5, 1.6].  Takes about a minute on 8 cores and 2 GiB.

    python tests/golden/make_l3_exact.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2605_25872_amd import inputs  # noqa: E402

L, SEED, SAMPLE = 3, 7, 0
T = inputs.temperatures(0.5, 1.6, 8)


def main() -> None:
    oracle.build()
    J = inputs.couplings(L, 1, seed=SEED, first_sample=SAMPLE)[0]
    res = oracle.exact_enumerate(L, J, 1.0 / T)
    out = {
        "what": "exact enumeration of one L=3 periodic 3D EA sample, Gaussian couplings",
        "generator": "paper_2605_25872_amd.inputs.couplings(L=3, n_samples=1, seed=7)",
        "L": L, "seed": SEED, "sample": SAMPLE,
        "T": T.tolist(),
        "e_mean": res["e"].tolist(),
        "e2_mean": res["e2"].tolist(),
        "ql_mean": res["ql"].tolist(),
        "pq": res["pq"].tolist(),
    }
    with open(os.path.join(HERE, "l3_exact.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
