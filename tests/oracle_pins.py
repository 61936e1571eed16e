"""Pins of the FP64 oracle against what mathematics fixes (not against itself).

Each pin returns a list of failure strings (empty = pass), so the same checks
run on the committed oracle and on deliberately broken copies of it (see the
mutation test): a plausible mistake anywhere in the oracle must trip at least
one pin.

Pins:
  direct1d / direct2d : recursive FFT == the DFT definition evaluated directly
  listing             : the bit-reversal + iterative butterfly form (Listing 1
                        reading) == the recursive form, every length 2 .. 2^14
  schedule            : one step of the iterative form pairs exactly the points
                        the eight-point example of Section 2.2 pairs (span 1,
                        2, 4), with the twiddle the step needs
  ramp8               : the closed-form DFT of the eight-point ramp
  closed forms        : delta, shifted delta, constant, cosine, one complex
                        exponential (fixes the exponent sign), rectangular grids
  invariants          : Parseval, linearity, circular shift <-> phase ramp,
                        Hermitian symmetry of real input, rows/columns order,
                        inverse round trip
  library             : numpy.fft (pocketfft), run as a black box
  matrix              : the separable matrix form F_M x F_N^T of the definition
  adjoint             : Re<F a, b> == Re<a, F^H b>, both directions
"""

from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    den = np.linalg.norm(b.ravel())
    num = np.linalg.norm((a - b).ravel())
    return num / den if den > 0 else num


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def pin_direct1d(o, tol=1e-12):
    fails = []
    rng = np.random.default_rng(11)
    for e in range(0, 7):
        n = 1 << e
        x = _rand(rng, n)
        for sign in (-1, 1):
            err = _rel(o.fft1d(x, sign), o.dft1d_direct(x, sign))
            if not err <= tol:
                fails.append("direct1d n=%d sign=%d err=%.3g" % (n, sign, err))
    return fails


def pin_direct2d(o, tol=1e-12, shapes=None):
    fails = []
    rng = np.random.default_rng(12)
    shapes = shapes or [(1, 1), (1, 8), (8, 1), (2, 4), (4, 2), (16, 8), (8, 32), (32, 32), (2, 64), (64, 4),
                        (64, 64)]
    for (M, N) in shapes:
        x = _rand(rng, (M, N))
        for sign in (-1, 1):
            err = _rel(o.fft2(x, sign), o.dft2d_direct(x, sign))
            if not err <= tol:
                fails.append("direct2d %dx%d sign=%d err=%.3g" % (M, N, sign, err))
    return fails


def pin_listing(o, tol=1e-13, max_log=14):
    fails = []
    rng = np.random.default_rng(13)
    for e in range(0, max_log + 1):
        n = 1 << e
        x = _rand(rng, n)
        for sign in (-1, 1):
            err = _rel(o.fft1d_listing(x, sign), o.fft1d(x, sign))
            if not err <= tol:
                fails.append("listing n=%d sign=%d err=%.3g" % (n, sign, err))
    for n in (2, 4, 8, 16):
        x = _rand(rng, n)
        err = _rel(o.fft1d_listing(x), o.dft1d_direct(x))
        if not err <= 1e-12:
            fails.append("listing-direct n=%d err=%.3g" % (n, err))
    return fails


def load_schedule():
    rows = np.loadtxt(os.path.join(GOLDEN, "fig2_schedule_8.txt"), dtype=np.int64, comments="#")
    return [(int(s), int(a), int(b)) for s, a, b in rows]


def pin_schedule(o):
    """A delta at the second point of a pair, run through one step alone, lands
    on exactly that pair: +w at the first point, -w at the second, where w is
    the step's twiddle exp(-2 pi i j / 2^(s+1)) for the pair's spectrum j."""
    fails = []
    n = 8
    for s, a, b in load_schedule():
        x = np.zeros(n, dtype=np.complex128)
        x[b] = 1.0
        y = o.fft1d_listing_steps(x, -1, permute=False, step_lo=s, step_hi=s)
        j = a % (1 << s)
        w = np.exp(-2j * np.pi * j / (1 << (s + 1)))
        want = np.zeros(n, dtype=np.complex128)
        want[a] = w
        want[b] = -w
        if not np.allclose(y, want, atol=1e-14, rtol=0):
            fails.append("schedule step=%d pair=(%d,%d)" % (s, a, b))
        x = np.zeros(n, dtype=np.complex128)
        x[a] = 1.0
        y = o.fft1d_listing_steps(x, -1, permute=False, step_lo=s, step_hi=s)
        want = np.zeros(n, dtype=np.complex128)
        want[a] = 1.0
        want[b] = 1.0
        if not np.allclose(y, want, atol=1e-14, rtol=0):
            fails.append("schedule-first step=%d pair=(%d,%d)" % (s, a, b))
    return fails


def pin_ramp8(o):
    fails = []
    ref = np.loadtxt(os.path.join(GOLDEN, "ramp8_dft.txt"), comments="#")
    want = ref[:, 1] + 1j * ref[:, 2]
    x = np.arange(8, dtype=np.float64).astype(np.complex128)
    for name, y in (("recursive", o.fft1d(x)), ("listing", o.fft1d_listing(x)),
                    ("fft2 1x8", o.fft2(x.reshape(1, 8))[0]), ("fft2 8x1", o.fft2(x.reshape(8, 1))[:, 0])):
        if not np.allclose(y, want, atol=1e-12, rtol=0):
            fails.append("ramp8 %s" % name)
    return fails


def pin_closed_forms(o, shapes=((8, 8), (4, 16), (32, 8), (1, 16), (16, 1), (64, 128))):
    fails = []
    for (M, N) in shapes:
        m = np.arange(M)[:, None]
        n = np.arange(N)[None, :]
        k, l = m, n
        # delta at the origin -> all ones
        x = np.zeros((M, N), dtype=np.complex128)
        x[0, 0] = 1
        if not np.allclose(o.fft2(x), np.ones((M, N)), atol=1e-12):
            fails.append("delta0 %dx%d" % (M, N))
        # shifted delta -> exp(-2 pi i (k p / M + l q / N))
        p, q = (M // 2 + 1) % M, (N // 3 + 1) % N
        x = np.zeros((M, N), dtype=np.complex128)
        x[p, q] = 1
        want = np.exp(-2j * np.pi * (k * p / M + l * q / N))
        if not np.allclose(o.fft2(x), want, atol=1e-12):
            fails.append("delta(p,q) %dx%d" % (M, N))
        # constant c -> c M N at (0, 0), zero elsewhere
        c = 0.75 - 0.25j
        want = np.zeros((M, N), dtype=np.complex128)
        want[0, 0] = c * M * N
        if not np.allclose(o.fft2(np.full((M, N), c)), want, atol=1e-11):
            fails.append("constant %dx%d" % (M, N))
        # one complex exponential exp(+2 pi i (k0 m / M + l0 n / N)) -> M N at (k0, l0)
        k0, l0 = (1 % M), (3 % N)
        x = np.exp(2j * np.pi * (k0 * m / M + l0 * n / N))
        want = np.zeros((M, N), dtype=np.complex128)
        want[k0, l0] = M * N
        if not np.allclose(o.fft2(x), want, atol=1e-10):
            fails.append("exponential %dx%d" % (M, N))
        # inverse of a single spike at (k0, l0) -> exp(+...) / (M N)
        X = np.zeros((M, N), dtype=np.complex128)
        X[k0, l0] = 1
        want = np.exp(2j * np.pi * (k0 * m / M + l0 * n / N)) / (M * N)
        if not np.allclose(o.ifft2(X), want, atol=1e-14):
            fails.append("inverse spike %dx%d" % (M, N))
        # cosine -> M N / 2 at (k0, l0) and (-k0, -l0)
        x = np.cos(2 * np.pi * (k0 * m / M + l0 * n / N)).astype(np.complex128)
        want = np.zeros((M, N), dtype=np.complex128)
        want[k0, l0] += M * N / 2
        want[(-k0) % M, (-l0) % N] += M * N / 2
        if not np.allclose(o.fft2(x), want, atol=1e-10):
            fails.append("cosine %dx%d" % (M, N))
    return fails


def pin_invariants(o, shapes=((16, 16), (8, 32), (64, 16), (128, 256))):
    fails = []
    rng = np.random.default_rng(14)
    for (M, N) in shapes:
        x = _rand(rng, (M, N))
        y = _rand(rng, (M, N))
        X = o.fft2(x)
        # Parseval: sum |X|^2 = M N sum |x|^2
        lhs, rhs = np.sum(np.abs(X) ** 2), M * N * np.sum(np.abs(x) ** 2)
        if not abs(lhs - rhs) <= 1e-12 * rhs:
            fails.append("parseval %dx%d" % (M, N))
        # linearity
        a, b = 0.3 - 1.2j, -2.0 + 0.5j
        if not _rel(o.fft2(a * x + b * y), a * X + b * o.fft2(y)) <= 1e-13:
            fails.append("linearity %dx%d" % (M, N))
        # circular shift by (p, q) multiplies by exp(-2 pi i (k p / M + l q / N))
        p, q = 3 % M, 5 % N
        k = np.arange(M)[:, None]
        l = np.arange(N)[None, :]
        ramp = np.exp(-2j * np.pi * (k * p / M + l * q / N))
        if not _rel(o.fft2(np.roll(x, (p, q), axis=(0, 1))), ramp * X) <= 1e-13:
            fails.append("shift %dx%d" % (M, N))
        # real input -> X[-k, -l] = conj X[k, l]
        Xr = o.fft2(x.real.astype(np.complex128))
        flip = np.roll(Xr[::-1, ::-1], (1, 1), axis=(0, 1))
        if not _rel(flip, np.conj(Xr)) <= 1e-13:
            fails.append("hermitian %dx%d" % (M, N))
        # columns-then-rows equals rows-then-columns
        if not _rel(o.fft2(np.ascontiguousarray(x.T)).T, X) <= 1e-13:
            fails.append("transpose %dx%d" % (M, N))
        # inverse round trip
        if not _rel(o.ifft2(X), x) <= 1e-14:
            fails.append("roundtrip %dx%d" % (M, N))
    return fails


def pin_library(o, shapes=((32, 64), (256, 128), (1024, 1024), (16384, 8), (4, 16384))):
    fails = []
    rng = np.random.default_rng(15)
    for (M, N) in shapes:
        x = _rand(rng, (M, N))
        if not _rel(o.fft2(x), np.fft.fft2(x)) <= 1e-12:
            fails.append("numpy fft2 %dx%d" % (M, N))
        if not _rel(o.ifft2(x), np.fft.ifft2(x)) <= 1e-12:
            fails.append("numpy ifft2 %dx%d" % (M, N))
    x = _rand(rng, (3, 16, 32))
    if not _rel(o.fft2(x), np.fft.fft2(x)) <= 1e-12:
        fails.append("numpy batched fft2")
    return fails


def _dft_matrix(n, sign):
    """F[k, m] = exp(sign 2 pi i (k m mod n) / n), the phase reduced in integers."""
    k = np.arange(n, dtype=np.int64)
    return np.exp(sign * 2j * np.pi * (np.outer(k, k) % n) / n)


def pin_matrix(o, shapes=((4, 8), (64, 32), (128, 256), (256, 256))):
    """The separable matrix form of the definition: X = F_M x F_N^T."""
    fails = []
    rng = np.random.default_rng(17)
    for (M, N) in shapes:
        x = _rand(rng, (M, N))
        for sign, scale in ((-1, 1.0), (1, 1.0 / (M * N))):
            ref = scale * (_dft_matrix(M, sign) @ x @ _dft_matrix(N, sign).T)
            err = _rel(o.fft2(x, sign, scale), ref)
            if not err <= 1e-12:
                fails.append("matrix %dx%d sign=%d err=%.3g" % (M, N, sign, err))
    return fails


def pin_adjoint(o, shapes=((16, 32), (64, 64))):
    fails = []
    rng = np.random.default_rng(16)
    for (M, N) in shapes:
        a = _rand(rng, (M, N))
        b = _rand(rng, (M, N))
        for d in (-1, 1):
            Fa = o.fft2(a, d, 1.0 if d == -1 else 1.0 / (M * N))
            lhs = np.vdot(b, Fa).real  # Re <F a, b>
            rhs = np.vdot(o.adjoint(b, d), a).real  # Re <a, F^H b>
            if not abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0):
                fails.append("adjoint %dx%d dir=%d" % (M, N, d))
    return fails


ALL_PINS = (pin_direct1d, pin_direct2d, pin_listing, pin_schedule, pin_ramp8, pin_closed_forms, pin_invariants,
            pin_library, pin_matrix, pin_adjoint)


def run_all(o, quick=False):
    fails = []
    for pin in ALL_PINS:
        if quick and pin is pin_library:
            fails += pin(o, shapes=((32, 64), (4, 16)))
        elif quick and pin is pin_direct2d:
            fails += pin(o, shapes=[(1, 8), (8, 1), (2, 4), (16, 8), (8, 32)])
        else:
            fails += pin(o)
    return fails
