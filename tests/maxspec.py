"""The largest operator spec the interface accepts, for tests on both sides."""
import random

from paper_2606_09551_amd import workloads as W

P = W.PredDesc


def max_int_spec(rnd: random.Random, n: int):
    """The interface's largest spec: 64 intervals, degree 3, 16 predicates of
    every kind, 16 comparison atoms, output bits up to 63 (some shared)."""
    N = 1 << n
    s = N // 2
    alpha = [0] + sorted(rnd.sample(range(1, N), 63)) + [N]
    coef = [[rnd.getrandbits(64) for _ in range(4)] for _ in range(64)]
    preds = [P(W.LT_UNSIGNED, 5 * i, thr=float(rnd.randint(1, N - 1)), negate=bool(i & 1)) for i in range(11)]
    preds += [P(W.LT_UNSIGNED, 63, thr=float(rnd.randint(1, N - 1))),
              P(W.LOWBITS_LT, 62, f_bits=n - 3, gamma=rnd.randint(1, (1 << (n - 3)) - 1)),
              P(W.MSB_SHIFT, 61, c=rnd.randint(1, N - 1)),
              P(W.LT_UNSIGNED, 0, thr=float(N)),            # sentinel C_N: constant 1, no atom
              P(W.LT_SIGNED, 60, thr=float(-s))]            # x < -N/2: constant 0, no atom
    return alpha, coef, preds
