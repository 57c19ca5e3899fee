"""Site decompositions on the device divide by truncating n * inv, with inv
= 1/d rounded up to the next binary64 (stored by the host) and no
correction step.  That equals floor(n/d) for 0 <= n < 2^31, 0 < d < 2^24
and n/d < 2^24, the bounds the extent checks at creation enforce.  Host
binary64 arithmetic is the same IEEE round-to-nearest product, so the rule
is checked here over divisors and quotients at the edges of those bounds."""
import math
import random


def quot(n, d, inv):
    return int(float(n) * inv)


def test_round_up_reciprocal_truncates_to_floor():
    rng = random.Random(7)
    ds = list(range(1, 2050)) + [rng.randrange(2, 1 << 24) for _ in range(1500)]
    ds += [(1 << 24) - 1, (1 << 23) + 1, 3 ** 15, 49, 98, 3 * 49 * 1024]
    for d in ds:
        inv = math.nextafter(1.0 / d, math.inf)
        qmax = min((1 << 24) - 1, ((1 << 31) - 1) // d)
        qs = {0, 1, qmax, max(qmax - 1, 0)} | {rng.randrange(0, qmax + 1) for _ in range(16)}
        # quotients at the top of binary64 binades, where rounding errors are largest
        qs |= {(1 << e) - 1 for e in range(1, 25) if (1 << e) - 1 <= qmax}
        for q in qs:
            for r in {0, 1, d // 2, d - 1}:
                n = q * d + r
                if r < d and n < (1 << 31):
                    assert quot(n, d, inv) == q, (n, d)


def test_nearest_reciprocal_alone_undershoots():
    # with 1/d rounded to nearest some exact quotients truncate one low
    # (49 * fl(1/49) < 1): the rounding up is what the helper relies on
    assert quot(49, 49, 1.0 / 49) == 0
    assert quot(49, 49, math.nextafter(1.0 / 49, math.inf)) == 1
