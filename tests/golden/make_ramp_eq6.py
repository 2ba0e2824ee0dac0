"""Writes ramp_eq6.txt: the band-limited ramp response evaluated from the paper's sinc form
(eq 6, h(n) = sinc(pi n)/2 - sinc^2(pi n / 2)/4, sinc(r) = sin(r)/r) for n = -12..12.

This evaluates the printed expression eq 6 directly; the oracle implements the simplified
case form eq 7, so the fixture checks that simplification.  Calls nothing from the oracle.
"""
import math
import os


def sinc(r):
    return 1.0 if r == 0 else math.sin(r) / r


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ramp_eq6.txt")
    with open(path, "w") as f:
        f.write("# n  h(n) from eq 6 (sinc form), written by make_ramp_eq6.py\n")
        for n in range(-12, 13):
            h = sinc(math.pi * n) / 2 - sinc(math.pi * n / 2) ** 2 / 4
            f.write(f"{n} {h:.17e}\n")


if __name__ == "__main__":
    main()
