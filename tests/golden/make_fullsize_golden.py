"""Writes fullsize_rsync.json: the oracle's round-synchronous Algorithm 3
(lower id keeps) and sequential First-Fit on the benchmark's full-size
graphs, as a digest per graph (sha256 of the input CSR and of the colour
array, K, recolouring rounds, conflicts, |L| per round).  Calls only the
seeded generators and oracle/; takes a few minutes on one core.

    python tests/golden/make_fullsize_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

CONFIGS = {
    "lattice26_200_perm": lambda: gg.lattice26(200, permute_seed=1505),
    "rmat22_shuffled": lambda: gg.rmat(22, 16, 0.57, 0.19, 0.19, seed=1505, shuffle_seed=1506),
}


def sha(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()


def main():
    out = {}
    for name, gen in CONFIGS.items():
        rp, ci = gen()
        r = oracle.rsync(rp, ci, tie="lower")
        _, kseq = oracle.seq_ff(rp, ci)
        out[name] = {"row_ptr_sha256": sha(rp), "col_idx_sha256": sha(ci), "n": len(rp) - 1, "nnz": len(ci),
                     "rsync_lower": {"colors_sha256": sha(r["colors"]), "K": r["K"], "rounds": r["rounds"],
                                     "conflicts": r["conflicts"], "L_sizes": [int(x) for x in r["L_sizes"]]},
                     "seq_ff_K": kseq}
        print(name, out[name]["rsync_lower"]["K"], out[name]["rsync_lower"]["rounds"], kseq, flush=True)
    with open(os.path.join(HERE, "fullsize_rsync.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
