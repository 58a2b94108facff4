"""Counter-based delay generator (oracle side).

Test infrastructure (oracle). Written from the published definitions, with
Python integers (arbitrary precision, reduced mod 2^64 explicitly).

- Sec. 5.1 (simulation of delays): at every time advancement a uniform number
  in [0, 1] is drawn for each PE boundary and matched against L bins of widths
  p_0 .. p_{L-1}; the bin index is the delay k. Draws are i.i.d. across PE
  boundaries, and a scheme with a uniform delay draws once per boundary per
  step.
- The uniform number is produced by hashing a counter with the SplitMix64
  finaliser of Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators" (OOPSLA 2014): golden-ratio increment 0x9E3779B97F4A7C15, then
  xor-shift 30 / multiply 0xBF58476D1CE4E5B9 / xor-shift 27 / multiply
  0x94D049BB133111EB / xor-shift 31.

Counter layout (a reading of this implementation; the paper names no
generator): draw(key, n, face) = mix(key + ((n << 32 | face) + 1) * G), where
face = p * 2 * ndim + 2 * axis + side, p the linear PE index with x fastest,
side 0 the low neighbour. The top 53 bits are compared with integer bin
thresholds THR[j] = floor(2^53 * (w_0 + .. + w_j) / (w_0 + .. + w_{L-1})) for
integer bin weights w_j proportional to p_j; the delay is the first j with
u53 < THR[j].
"""

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z):
    """SplitMix64 output finaliser on a 64-bit integer."""
    z &= MASK64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & MASK64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & MASK64
    z ^= z >> 31
    return z


def splitmix64_stream(seed, count):
    """The plain SplitMix64 sequence: state += G, output mix(state)."""
    out = []
    state = seed & MASK64
    for _ in range(count):
        state = (state + GOLDEN) & MASK64
        out.append(mix64(state))
    return out


def draw(key, n, face):
    """64-bit hash of the counter (n, face) under ``key``."""
    ctr = ((n << 32) | face) + 1
    return mix64((key + ctr * GOLDEN) & MASK64)


def thresholds(L, weights=None):
    """Cumulative 53-bit bin thresholds for delays 0..L-1 (Sec. 5.1 bins)."""
    if weights is None:
        weights = [1] * L
    if len(weights) != L or any(w < 0 for w in weights) or sum(weights) == 0:
        raise ValueError("need L non-negative integer bin weights with a positive sum")
    total = sum(weights)
    thr = []
    cum = 0
    for w in weights:
        cum += w
        thr.append((cum << 53) // total)
    return thr


def bin_delay(u53, thr):
    for j, t in enumerate(thr):
        if u53 < t:
            return j
    raise AssertionError("u53 must be below 2^53")


def raw_delay(key, n, face, thr):
    """Delay k~ in [0, L-1] before the start-up clamp."""
    return bin_delay(draw(key, n, face) >> 11, thr)


def clamp_startup(k, n, T):
    """No level before t = 0 exists: k = min(k~, max(0, n - T + 1)).

    With this clamp the oldest level touched, n - k - (T - 1), is never
    negative. (A reading: the paper starts its runs without discussing the
    first steps.)"""
    return min(k, max(0, n - T + 1))


def ensemble_key(seed_base, i):
    """Independent key of ensemble member i."""
    return mix64((seed_base + (i + 1) * GOLDEN) & MASK64)
