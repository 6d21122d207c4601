"""Writes the stored expected values that come from the oracle (not from the
paper).  Calls only oracle/ and the standard library.

    python tests/golden/make_golden.py
"""
import itertools
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fitness as F  # noqa: E402


def search_box(f_star=30.0, m_lo=1.0, m_hi=3.0, n=401):
    ms = [m_lo + (m_hi - m_lo) * i / (n - 1) for i in range(n)]
    t0s, t15s = [], []
    for a, b in itertools.product(ms, ms):
        t0, t15 = F.chirp_times_from_masses(a, b, f_star)
        t0s.append(t0)
        t15s.append(t15)
    return dict(f_star_hz=f_star, mass_range_msun=[m_lo, m_hi],
                tau0_s=[min(t0s), max(t0s)], tau15_s=[min(t15s), max(t15s)],
                note="extremes over a 401x401 grid of the mass square; written by oracle.fitness.chirp_times_from_masses")


if __name__ == "__main__":
    with open(os.path.join(HERE, "search_box_30hz.json"), "w") as fh:
        json.dump(search_box(), fh, indent=2)
        fh.write("\n")
