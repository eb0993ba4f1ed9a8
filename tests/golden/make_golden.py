"""Write tests/golden/*.json from the CPU oracle only (no HIP code is imported).

For each named workload this stores E0 = <C|H|C> (oracle double loop) and, when
the oracle can run the whole search in a few minutes, the exact facts of its
result (Alg. 2 with the score of Eq. (1)): number of pairs, number of
candidates, SHA-256 of the candidate keys / numerators / scores in ascending
key order, SHA-256 of the top-k keys and scores in selection order, the
first entries of the top-k as hex floats, and the second-order energy
sum_a N_a^2 / (E0 - H_aa) over the candidates (compensated sum) with the sum
of the absolute values of its terms.

    python tests/golden/make_golden.py 8e12o 16e20o 24e30o
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import asci_synth as syn  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
FULL_SEARCH = {"8e12o", "16e20o"}  # the oracle's full search fits in minutes


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(names):
    oracle.build(force=False)
    for name in names:
        t0 = time.time()
        c = syn.workload(name)
        n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
        out = {
            "workload": name,
            "source": "oracle (CPU, plain C); Alg. 2 and Eq. (1) of the paper",
            "norb": n, "nalpha": na, "nbeta": nb, "ndets": int(len(c["coeffs"])), "k": c["k"],
            "seed": c["seed"],
        }
        E0 = oracle.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
        out["E0"] = E0.hex()
        out["pairs_closed_form"] = int(len(c["coeffs"]) * oracle.sd_count(n, na, nb))
        if name in FULL_SEARCH:
            r = oracle.search_all(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0)
            idx = oracle.topk_index(r["keys"], r["score"], c["k"])
            tk, ts = r["keys"][idx], r["score"][idx]
            out.update({
                "npairs": int(r["npairs"]),
                "ncandidates": int(len(r["score"])),
                "cand_keys_sha256": sha(r["keys"]),
                "cand_num_sha256": sha(r["num"]),
                "cand_score_sha256": sha(r["score"]),
                "topk_count": int(len(idx)),
                "topk_keys_sha256": sha(tk),
                "topk_scores_sha256": sha(ts),
                "topk_head": [[int(a), int(b), float(s).hex()] for (a, b), s in zip(tk[:16], ts[:16])],
                "kth_abs_score": float(abs(ts[-1])).hex(),
            })
            e2, ncand, s2 = oracle.pt2(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, with_abs=True)
            out["pt2"] = e2.hex()
            out["pt2_abs_terms"] = s2.hex()
        out["oracle_seconds"] = round(time.time() - t0, 1)
        with open(os.path.join(HERE, "search_%s.json" % name), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "done in %.1fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["8e12o", "16e20o", "24e30o"])
