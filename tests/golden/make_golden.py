"""Write tests/golden/*.json from the CPU oracle only (no HIP code is imported).

For each named workload this stores E0 = <C|H|C> (oracle double loop) and the
facts of the oracle's search result (Alg. 2 with the score of Eq. (1)):

- number of pairs and of candidates; for the workloads whose candidates fit in
  memory, SHA-256 of the candidate keys in ascending key order (exact: the
  candidate set is combinatorial) and, for information only, of the
  numerators and scores;
- the top-k under the score tolerance (oracle_score_tol): the keys every
  evaluation order within the tolerance must select (count and SHA-256 of
  their sorted keys), the ambiguous candidates near the k-th value (keys,
  scores, tolerances), and bounds on the k-th |A| of any such selection;
- the first entries of the top-k with their tolerances (hex floats);
- the second-order energy sum_a N_a A_a (Neumaier sums), sum |N_a A_a| and the
  sum of per-term tolerances.

The search runs in the oracle's bucketed mode (the same bits as the flat
search, threaded over target buckets).  For 24e30o only each bucket's best
k + k/10 candidates are kept and merged; the bands then also account for every
dropped candidate through the largest |A| + tol among them.

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
ALL_CANDIDATES = {"8e12o", "16e20o"}  # every candidate fits in host memory
HEAD = 64


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def hexes(x):
    return [float(v).hex() for v in x]


def by_key(r):
    o = np.argsort(oracle.key_codes(r["keys"]), kind="stable")
    return {f: (v[o] if isinstance(v, np.ndarray) else v) for f, v in r.items()}


def select(r, k):
    """(|A| desc, key asc) order of the candidates of r, first k."""
    return oracle.topk_index(r["keys"], r["score"], k)


def merged_search(c, E0, k, nbuckets=256, group=16):
    """Bucketed search keeping each bucket's best k + k/10: (pool, stats, largest U dropped)."""
    n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
    keep = k + k // 10
    pool, drop_up = None, 0.0
    tot = {"candidates": 0, "npairs": 0, "pt2_parts": [], "pt2_abs": 0.0, "pt2_tol": 0.0}
    for b0 in range(0, nbuckets, group):
        t0 = time.time()
        r, st = oracle.search_buckets(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, nbuckets=nbuckets,
                                      buckets=(b0, min(nbuckets, b0 + group)), keep_top=keep)
        tot["candidates"] += st["candidates"]
        tot["npairs"] += st["npairs"]
        tot["pt2_parts"].append(st["pt2"])
        tot["pt2_abs"] += st["pt2_abs"]
        tot["pt2_tol"] += st["pt2_tol"]
        drop_up = max(drop_up, st["max_drop_upper"])
        pool = r if pool is None else {f: np.concatenate([pool[f], r[f]]) if isinstance(r[f], np.ndarray) else r[f]
                                       for f in r}
        if len(pool["score"]) > keep:
            idx = select(pool, len(pool["score"]))
            out = idx[keep:]
            drop_up = max(drop_up, float((np.abs(pool["score"][out]) + pool["tol"][out]).max()))
            pool = {f: (v[idx[:keep]] if isinstance(v, np.ndarray) else v) for f, v in pool.items()}
        print("  buckets %d-%d: %d candidates so far, %.0fs" % (b0, b0 + group, tot["candidates"], time.time() - t0),
              flush=True)
    return pool, tot, drop_up


def topk_facts(r, k, outside_upper=0.0):
    idx = select(r, k)
    sure_in, amb, outside_ok = oracle.topk_bands(r["keys"], r["score"], r["tol"], k, outside_upper)
    if not outside_ok:
        raise RuntimeError("dropped candidates could reach the top k: keep more per bucket")
    chosen = np.zeros(len(r["score"]), bool)
    chosen[idx] = True
    assert not (sure_in & ~chosen).any() and not (chosen & ~sure_in & ~amb).any()
    sk = np.sort(oracle.key_codes(r["keys"][sure_in]))
    a = np.abs(r["score"])
    L, U = np.sort(a - r["tol"])[::-1], np.sort(a + r["tol"])[::-1]
    m = min(k, len(a))
    ai = np.nonzero(amb)[0]
    ai = ai[np.argsort(oracle.key_codes(r["keys"][ai]), kind="stable")]
    head = idx[:HEAD]
    return {
        "topk_count": int(len(idx)),
        "topk_keys_sha256_oracle_order": sha(r["keys"][idx]),
        "sure_count": int(sure_in.sum()),
        "sure_keys_sha256": sha(sk),
        "ambiguous": [[int(r["keys"][j, 0]), int(r["keys"][j, 1]), float(r["score"][j]).hex(),
                       float(r["tol"][j]).hex()] for j in ai],
        "kth_abs_score": float(a[idx[-1]]).hex() if m else None,
        "kth_lo": float(L[m - 1]).hex() if m else None,
        "kth_hi": float(U[m - 1]).hex() if m else None,
        "topk_head": [[int(r["keys"][j, 0]), int(r["keys"][j, 1]), float(r["score"][j]).hex(),
                       float(r["tol"][j]).hex()] for j in head],
    }


def main(names):
    oracle.build(force=False)
    for name in names:
        t0 = time.time()
        c = syn.workload(name)
        n, na, nb, k = c["norb"], c["nalpha"], c["nbeta"], c["k"]
        out = {
            "workload": name,
            "source": "oracle (CPU, plain C); Alg. 2 and Eq. (1) of the paper; scores compared within "
                      "oracle_score_tol",
            "norb": n, "nalpha": na, "nbeta": nb, "ndets": int(len(c["coeffs"])), "k": k, "seed": c["seed"],
        }
        E0 = oracle.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
        out["E0"] = E0.hex()
        out["pairs_closed_form"] = int(len(c["coeffs"]) * oracle.sd_count(n, na, nb))
        print(name, "E0 done in %.1fs" % (time.time() - t0), flush=True)
        if name in ALL_CANDIDATES:
            r, st = oracle.search_buckets(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, nbuckets=64)
            r = by_key(r)
            relaxed = int((r["tol"] > 1.000001e-12 * np.abs(r["score"])).sum())
            out.update({
                "npairs": int(st["npairs"]),
                "ncandidates": int(st["candidates"]),
                "cand_keys_sha256": sha(r["keys"]),
                "cand_num_sha256_info": sha(r["num"]),
                "cand_score_sha256_info": sha(r["score"]),
                "relaxed_band": relaxed,
            })
            out.update(topk_facts(r, k))
            pt2 = (st["pt2"], st["pt2_abs"], st["pt2_tol"])
        else:
            pool, tot, drop_up = merged_search(c, E0, k)
            out.update({"npairs": int(tot["npairs"]), "ncandidates": int(tot["candidates"]),
                        "largest_dropped_upper": float(drop_up).hex()})
            out.update(topk_facts(pool, k, outside_upper=drop_up))
            import math
            pt2 = (math.fsum(tot["pt2_parts"]), tot["pt2_abs"], tot["pt2_tol"])
        out["pt2"] = float(pt2[0]).hex()
        out["pt2_abs_terms"] = float(pt2[1]).hex()
        out["pt2_term_tol"] = float(pt2[2]).hex()
        out["oracle_seconds"] = round(time.time() - t0, 1)
        with open(os.path.join(HERE, "search_%s.json" % name), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "done in %.1fs: %d candidates, %d sure, %d ambiguous" % (
            time.time() - t0, out["ncandidates"], out["sure_count"], len(out["ambiguous"])), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["8e12o", "16e20o", "24e30o"])
