"""Writes sim_medium5k.json: similarity counts of the 5,000-class synthetic
system under each threshold, computed by the CPU oracle only (all pairs, about
three minutes single-threaded). Run from the repository root:
    python tests/golden/make_similarity_golden.py
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
from oracle import oracle as O  # noqa: E402
from paper_1308_4011_amd import synth  # noqa: E402


def main():
    s = synth.medium(5000)
    pairs = O.similarity_pairs(s)
    m1, m2, inter, union = pairs
    out = {"cite": "Sec. II-A (Jaccard similarity of methods), Sec. III-A and its footnote (average threshold); "
                   "written by tests/golden/make_similarity_golden.py from the CPU oracle",
           "workload": "synth.medium(5000)", "n_methods": int(s.n_methods), "n_nonzero": int(len(m1)),
           "thresholds": {}}
    for name, th in (("nonzero", O.SIM_NONZERO), ("above_avg", O.SIM_ABOVE_AVG),
                     ("above_avg_nz", O.SIM_ABOVE_AVG_NZ)):
        avg = None if th == O.SIM_NONZERO else O.similarity_average(s.n_methods, inter, union, th)
        keep = O.similarity_kept(s.n_methods, inter, union, th)
        cm, ct = O.similar_candidates(s, th, pairs)
        out["thresholds"][name] = {
            "average": None if avg is None else [str(avg.numerator), str(avg.denominator)],
            "n_high": int(keep.sum()), "n_candidates": int(len(cm)),
            # a fixed sample of the candidate list (positions and entries)
            "sample_pos": np.linspace(0, max(len(cm) - 1, 0), 64).astype(int).tolist(),
            "sample": [[int(cm[k]), int(ct[k])] for k in np.linspace(0, max(len(cm) - 1, 0), 64).astype(int)],
        }
        print(name, out["thresholds"][name]["n_high"], out["thresholds"][name]["n_candidates"], flush=True)
    with open(os.path.join(os.path.dirname(__file__), "sim_medium5k.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
