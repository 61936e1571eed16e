"""Writes the closed-form fixtures of this folder (no FFT code is used).

ramp8_dft.txt: forward DFT (exponent sign -1) of x[m] = m, m < 8. For k != 0,
sum_m m w^m with w = exp(-2 pi i k/N) equals N / (w - 1), which simplifies to
-N/2 + i (N/2) cot(pi k/N); for k = 0 the sum is N (N - 1) / 2.

fig2_schedule_8.txt: for the eight-point radix-2 example of Section 2.2
(Fig. 2), step s (s = 0, 1, 2) pairs point p with point p + 2**s, for every p
whose bit s is zero. Each line: step, first point, second point.
"""

import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    N = 8
    with open(os.path.join(HERE, "ramp8_dft.txt"), "w") as f:
        f.write("# k re im : forward DFT of x[m] = m, N = 8, closed form -N/2 + i (N/2) cot(pi k/N)\n")
        for k in range(N):
            if k == 0:
                re, im = N * (N - 1) / 2.0, 0.0
            else:
                re, im = -N / 2.0, (N / 2.0) / math.tan(math.pi * k / N)
            f.write("%d %.17g %.17g\n" % (k, re, im))
    with open(os.path.join(HERE, "fig2_schedule_8.txt"), "w") as f:
        f.write("# step first second : radix-2 pairs of the 8-point example, span 2**step\n")
        for s in range(3):
            for p in range(N):
                if not (p >> s) & 1:
                    f.write("%d %d %d\n" % (s, p, p + (1 << s)))


if __name__ == "__main__":
    main()
