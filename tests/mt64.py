"""The 64-bit Mersenne Twister of Matsumoto and Nishimura with the parameters of
the C++ standard's std::mt19937_64, written out from its published definition,
for reproducing on the host the shuffles that the library draws from it."""

_N, _M = 312, 156
_MASK = (1 << 64) - 1
_UPPER, _LOWER = 0xFFFFFFFF80000000, 0x7FFFFFFF


def mt19937_64(seed):
    """Generator of the engine's 64-bit outputs for the given seed."""
    mt = [seed & _MASK]
    for i in range(1, _N):
        mt.append((6364136223846793005 * (mt[-1] ^ (mt[-1] >> 62)) + i) & _MASK)
    k = _N
    while True:
        if k >= _N:
            for i in range(_N):
                x = (mt[i] & _UPPER) | (mt[(i + 1) % _N] & _LOWER)
                xa = x >> 1
                if x & 1:
                    xa ^= 0xB5026F5AA96619E9
                mt[i] = mt[(i + _M) % _N] ^ xa
            k = 0
        y = mt[k]
        k += 1
        y ^= (y >> 29) & 0x5555555555555555
        y ^= (y << 17) & 0x71D67FFFEDA60000
        y ^= (y << 37) & 0xFFF7EEE000000000
        y ^= y >> 43
        yield y & _MASK


def shuffled_epochs(n, epochs, seed):
    """Sample orders of the training epochs: one generator for all epochs, each
    epoch a Fisher-Yates pass (k from n - 1 down to 1, j = word mod (k + 1))
    over the previous epoch's order."""
    g = mt19937_64(seed)
    order = list(range(n))
    out = []
    for _ in range(epochs):
        for k in range(n - 1, 0, -1):
            j = next(g) % (k + 1)
            order[k], order[j] = order[j], order[k]
        out.append(list(order))
    return out
