"""Writes the stored expected values under tests/golden/.

Only mpmath (50 significant digits) is used: no value here comes from
either evaluator.

worked_example.txt -- f(x) = (sin x + x)^2, the example function of the
paper's Fig. 2 and of its generated-kernel listing (three atomic
operations: sin, add, multiply, with work slot 1 reused in place).
"""

import os

import mpmath

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    mpmath.mp.dps = 50
    xs = ["0", "0.5", "1", "pi/2", "pi", "-2", "1e-8", "3.75"]
    lines = ["# x (C99 hex float, an exact double)  f(x)=(sin x + x)^2 at 40 digits",
             "# source: paper Fig. 2 / generated-kernel listing example function"]
    for s in xs:
        if s == "pi/2":
            x = float(mpmath.pi / 2)
        elif s == "pi":
            x = float(mpmath.pi)
        else:
            x = float(s)
        xm = mpmath.mpf(x)  # the exact double
        f = (mpmath.sin(xm) + xm) ** 2
        lines.append(f"{x.hex()} {mpmath.nstr(f, 40, min_fixed=-100, max_fixed=100)}")
    with open(os.path.join(HERE, "worked_example.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
