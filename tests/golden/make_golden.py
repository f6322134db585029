"""Writes the stored expected values under tests/golden/ from the CPU
reference only (oracle/).  Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import nystrom, rskel  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    with open(os.path.join(HERE, "self_cell_laplace.txt"), "w") as fh:
        fh.write("# n  int_{cell} (1/2pi) log|y| dy for the cell of side h = 1/n\n")
        fh.write("# closed form of the self-cell term (Nystrom diagonal, Sec. 5 general formulation)\n")
        for n in (32, 64, 128, 256, 512, 1024):
            fh.write(f"{n} {nystrom.self_cell_laplace(1.0 / n):.17e}\n")
    with open(os.path.join(HERE, "levels.txt"), "w") as fh:
        fh.write("# nx ny leaf m | per depth from the root: box shapes and sizes\n")
        fh.write("# depth ax ay count k r p  (k = |I^sk|, r = |I^rs|, p = |Z proxy|; Sec. 3.1)\n")
        for (nx, ny, leaf, m) in [(64, 64, 8, 2), (256, 256, 8, 2), (40, 24, 8, 2), (37, 37, 8, 2),
                                  (64, 64, 8, 1), (32, 32, 8, 3)]:
            root, levels = rskel.index_sets(nx, ny, leaf, m)
            fh.write(f"grid {nx} {ny} {leaf} {m}\n")
            for depth, lev in enumerate(levels):
                shapes = {}
                for b in lev:
                    key = (b.shape, len(b.sk), len(b.rs))
                    shapes[key] = shapes.get(key, 0) + 1
                for ((ax, ay), k, r), cnt in sorted(shapes.items()):
                    p = (ax + 2 * m) * (ay + 2 * m) - ax * ay
                    fh.write(f"{depth} {ax} {ay} {cnt} {k} {r} {p}\n")


if __name__ == "__main__":
    main()
