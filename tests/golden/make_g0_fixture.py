"""Write g0_rmat10_counts.json: oracle counts and traversed-edge credits for the
scale-10 R-MAT workload (edge factor 16, generator seed 1, 32 seeds drawn with
seed 7) at k = 1, 2, 3, 6.  Calls only the input generator and the oracle."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402


def main():
    el = graphgen.rmat(10, 16, seed=1)
    seeds = graphgen.draw_seeds(el, 32, seed=7)
    g = oracle.OracleGraph.from_edgelist(el)
    out = {"graph": "rmat scale 10, edge factor 16, a/b/c = 0.57/0.19/0.19, generator seed 1, undirected",
           "seeds": seeds.tolist(), "counts": {}, "te": {}}
    for k in (1, 2, 3, 6):
        c, te = g.count(seeds, k)
        out["counts"][str(k)] = c.tolist()
        out["te"][str(k)] = te.tolist()
    with open(os.path.join(HERE, "g0_rmat10_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
