"""Writes nearest_index_table.txt: for the 640x480 image and the 40x30 feature
map, the feature-map row chosen for every image row u and column for every
image column v by Eq. (target_continuous): round(u (Hf-1)/max(H-1,1)).

Exact rational arithmetic from the standard library; round() on a Fraction is
round-half-to-even.  Run: python tests/golden/make_nearest_table.py
"""
import os
from fractions import Fraction

H, W, HF, WF = 480, 640, 30, 40


def main():
    rows = [round(Fraction(u * (HF - 1), max(H - 1, 1))) for u in range(H)]
    cols = [round(Fraction(v * (WF - 1), max(W - 1, 1))) for v in range(W)]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "nearest_index_table.txt")
    with open(path, "w") as f:
        f.write(f"# Eq. (target_continuous), H={H} W={W} Hf={HF} Wf={WF}; line 1 rows, line 2 cols\n")
        f.write(" ".join(map(str, rows)) + "\n")
        f.write(" ".join(map(str, cols)) + "\n")


if __name__ == "__main__":
    main()
