"""Writes example2_*.json: the oracle's Example 2 (Section 4.2) errors.

Runs only the CPU oracle (float64), about 20 minutes for the 128 x 128 case:
    python tests/golden/make_example2.py 128 10
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from tests.paper_examples import example2  # noqa: E402

if __name__ == "__main__":
    N = int(sys.argv[1]) if len(sys.argv) > 1 else 128
    c = float(sys.argv[2]) if len(sys.argv) > 2 else 10.0
    E = example2(N, c=c)
    out = dict(example=2, N=N, c=c, T=0.2, phi=1.0, beta=1.0, tol=1e-12, errors=E,
               paper_bound=1.91e-3, source="oracle (float64), tests/paper_examples.example2")
    with open(os.path.join(HERE, f"example2_N{N}_c{int(c)}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
