"""Writes dft_pairs.json: closed-form DFT pairs from Eq. (1) of the tcFFT paper,
worked out by hand and typed in here with ``math`` only (no repository code
computes them).  Run: python tests/golden/make_dft_pairs.py"""
import json
import math
import os

r2 = math.sqrt(2.0)
pairs = [
    {"name": "ramp4", "cite": "Eq. (1); X[k]=sum_n (n+1) W_4^{nk}",
     "x": [[1, 0], [2, 0], [3, 0], [4, 0]], "X": [[10, 0], [-2, 2], [-2, 0], [-2, -2]]},
    {"name": "tone4_f1", "cite": "Eq. (1); x[n]=exp(+2 pi i n/4) -> 4 delta[k-1]",
     "x": [[1, 0], [0, 1], [-1, 0], [0, -1]], "X": [[0, 0], [4, 0], [0, 0], [0, 0]]},
    {"name": "rect8_half",
     "cite": "Eq. (1); rectangular pulse of width 4 in N=8: X[k]=sum_{n<4} W_8^{nk}",
     "x": [[1, 0]] * 4 + [[0, 0]] * 4,
     "X": [[4, 0], [1, -(1 + r2)], [0, 0], [1, -(r2 - 1)], [0, 0], [1, (r2 - 1)], [0, 0],
           [1, (1 + r2)]]},
    {"name": "alternating8", "cite": "Eq. (1); x[n]=(-1)^n in N=8 -> 8 delta[k-4]",
     "x": [[(-1) ** n, 0] for n in range(8)], "X": [[0, 0]] * 4 + [[8, 0]] + [[0, 0]] * 3},
    {"name": "delta2_16",
     "cite": "Eq. (1); x[n]=delta[n-2] in N=16 -> X[k]=W_16^{2k}=exp(-i pi k/4)",
     "x": [[1 if n == 2 else 0, 0] for n in range(16)],
     "X": [[math.cos(-math.pi * k / 4), math.sin(-math.pi * k / 4)] for k in range(16)]},
]

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dft_pairs.json")
    json.dump({"about": "Closed-form DFT pairs (forward transform, sign -1) used as fixtures "
               "for the FP64 oracle. Each value follows from Eq. (1) of the tcFFT paper by "
               "hand; none is produced by any code path of this repository.",
               "pairs": pairs}, open(out, "w"), indent=1)
