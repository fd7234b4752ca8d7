"""Write the printed sparsity coordinates of the first panel of Fig. KKTsystemOPF
(the 78x78 symmetric KKT of a 9-bus OPF in the ordering of Eq. SCOPFhessianSymmetric,
section 2.1) to a small text fixture.

The figure's panel prints every nonzero as an "x y" pair (1-based, nz = 576).
This script only copies those printed numbers; it computes nothing.
Run once with the LaTeX source of the paper as the argument:
    python tests/golden/extract_e1_pattern.py <paper source .tex/.md>
"""
import os
import re
import sys

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "e1_case9_kkt_pattern.txt")


def main(src):
    lines = open(src, encoding="utf-8").read().splitlines()
    label = next(i for i, l in enumerate(lines) if r"\label{fig:KKTsystemOPF}" in l)
    start = max(i for i in range(label) if lines[i].startswith(r"\begin{figure}"))
    ax0 = next(i for i in range(start, label) if r"\begin{axis}" in lines[i])
    ax1 = next(i for i in range(ax0, label) if r"\end{axis}" in lines[i])
    nz_label = None
    pairs = []
    pat = re.compile(r"^\s*(\d+)\s+(\d+)\s*\\\\\s*$")
    for l in lines[ax0:ax1]:
        m = re.search(r"xlabel=\{nz = (\d+)\}", l)
        if m:
            nz_label = int(m.group(1))
        m = pat.match(l)
        if m:
            pairs.append((int(m.group(1)), int(m.group(2))))
    with open(OUT, "w") as f:
        f.write("# Fig. KKTsystemOPF, first panel (section 2.1, Eq. SCOPFhessianSymmetric ordering)\n")
        f.write("# 9-bus OPF KKT, 78x78: x=(theta1..9, V1..9, Pg1..3, Qg1..3) rows 1-24,\n")
        f.write("# slacks 25-42, lambda_E 43-60 (P-balance 43-51, Q-balance 52-60), lambda_I 61-78.\n")
        f.write("# Coordinates copied verbatim from the figure's plot table, 1-based.\n")
        f.write(f"# printed nz = {nz_label}; pairs = {len(pairs)}\n")
        for a, b in pairs:
            f.write(f"{a} {b}\n")
    print(f"wrote {OUT}: {len(pairs)} pairs, printed nz = {nz_label}")


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: extract_e1_pattern.py <paper source>")
    sys.exit(main(sys.argv[1]))
