"""The near-contact force probes along the lattice direction closest to
n = -G/|G| (largest (c.n)/|c|, exact ties to the smaller |c|^2, then to the
lexicographically larger (c_x, c_y, c_z)).  The GPU kernel scores only the
candidates whose non-zero components carry the signs of n, arguing that no
other candidate can reach or tie the winner after rounding.  This test checks
that argument in FP32 arithmetic (the kernel's, same operation order): the
reduced search against the full search over every direction of D3Q19 and
D3Q27, on random vectors and on vectors built to produce exact ties, zero
components and components far below the others.  It checks the selection
rule the kernel implements, not the kernel's code (GPU parity covers that)."""
import itertools

import numpy as np
import pytest

f32 = np.float32
I2, I3 = f32(0.70710678118654752440), f32(0.57735026918962576451)


def _dirs(q):
    out = []
    for s in (1, 2, 3):
        for cx in (1, 0, -1):
            for cy in (1, 0, -1):
                for cz in (1, 0, -1):
                    if cx * cx + cy * cy + cz * cz != s or (q == 19 and s == 3):
                        continue
                    out.append((cx, cy, cz, s))
    return out


def _key(cx, cy, cz):
    return 13 + 9 * cx + 3 * cy + cz


def full_search(G, q):
    Gx, Gy, Gz = (G[:, k].astype(f32) for k in range(3))
    best = np.full(len(G), -np.inf, dtype=f32)
    key = np.full(len(G), -1)
    for cx, cy, cz, s in _dirs(q):
        inv = {1: f32(1.0), 2: I2, 3: I3}[s]
        dot = (f32(cx) * Gx + f32(cy) * Gy) + f32(cz) * Gz  # products are exact
        score = (-dot) * inv
        take = score > best
        best = np.where(take, score, best)
        key = np.where(take, _key(cx, cy, cz), key)
    return key


def octant_search(G, q):
    Gx, Gy, Gz = (G[:, k].astype(f32) for k in range(3))
    ax, ay, az = np.abs(Gx), np.abs(Gy), np.abs(Gz)
    kx = np.where(Gx > 0, -9, 9)
    ky = np.where(Gy > 0, -3, 3)
    kz = np.where(Gz > 0, -1, 1)

    def better(score, k, best, bkey):
        take = (score > best) | ((score == best) & (k > bkey))
        return np.where(take, score, best), np.where(take, k, bkey)

    b1, k1 = ax, 13 + kx
    b1, k1 = better(ay, 13 + ky, b1, k1)
    b1, k1 = better(az, 13 + kz, b1, k1)
    b2, k2 = (ax + ay) * I2, 13 + kx + ky
    b2, k2 = better((ax + az) * I2, 13 + kx + kz, b2, k2)
    b2, k2 = better((ay + az) * I2, 13 + ky + kz, b2, k2)
    key = np.where(b2 > b1, k2, k1)
    if q == 27:
        b3 = ((ax + ay) + az) * I3
        key = np.where(b3 > np.maximum(b1, b2), 13 + kx + ky + kz, key)
    return key


def _cases(seed):
    rng = np.random.default_rng(seed)
    n = 40000
    parts = [rng.standard_normal((n, 3))]
    # exact ties: equal magnitudes with random signs, in every pattern
    mag = rng.uniform(0.1, 2.0, (n, 1))
    sign = rng.choice([-1.0, 1.0], (n, 3))
    pattern = np.array(list(itertools.product([0.0, 1.0], repeat=3)))[rng.integers(0, 8, n)]
    parts.append(mag * sign * pattern)
    # two equal components and a third from another scale
    t = mag * sign
    t[:, 2] *= rng.choice([0.0, 1e-9, 0.5, 1.0, 1.4142135, 2.0, 1e6], n)
    parts.append(t[:, rng.permutation(3)])
    # components far below the others, negative zeros
    w = rng.standard_normal((n, 3)) * np.array([1.0, 1e-8, 1e-30])
    parts.append(w[:, rng.permutation(3)])
    parts.append(np.array([[-0.0, 1.0, 0.0], [0.0, -0.0, -1.0], [1.0, -1.0, 1.0], [-1.0, -1.0, -1.0]]))
    # exact ties between an axis and a diagonal: |G_x| = (|G_x| + |G_y|)/sqrt 2
    # after rounding, found among a few ulps around |G_y| = (sqrt 2 - 1)|G_x|
    a = rng.uniform(0.5, 2.0, 4000).astype(f32)
    b0 = (a * f32(np.sqrt(2.0) - 1.0)).astype(f32)
    for step in range(-4, 5):
        b = np.nextafter(b0, np.where(step > 0, np.inf, -np.inf).astype(f32)) if step else b0
        for _ in range(abs(step) - 1):
            b = np.nextafter(b, np.where(step > 0, np.inf, -np.inf).astype(f32))
        tie = ((a + b) * I2 == a)
        g = np.stack([-a[tie], -b[tie], np.zeros(tie.sum(), f32)], axis=1)
        parts.append(g[:, rng.permutation(3)] * rng.choice([-1.0, 1.0], (tie.sum(), 3)))
    G = np.concatenate(parts).astype(f32)
    return G[np.any(G != 0, axis=1)]


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("seed", [0, 1])
def test_octant_search_equals_full_search(q, seed):
    G = _cases(seed)
    full, red = full_search(G, q), octant_search(G, q)
    bad = np.nonzero(full != red)[0]
    assert bad.size == 0, (G[bad[:5]], full[bad[:5]], red[bad[:5]])


def test_full_search_tie_rules():
    """The canonical order itself: on an exact tie the shorter direction wins,
    then the lexicographically larger one."""
    G = np.array([[-1.0, -1.0, 0.0],   # n = (1,1,0): the diagonal beats both axes
                  [1.0, 0.0, -1.0],    # n = (-1,0,1): (0,0,1) and (-1,0,0) tie, (-1,0,1) wins
                  [-2.0, -1.0, -1.0],  # D3Q19: (1,1,0) and (1,0,1) tie, (1,1,0) is larger
                  [0.0, 0.0, 3.0]], dtype=f32)
    k19 = full_search(G, 19)
    assert list(k19) == [_key(1, 1, 0), _key(-1, 0, 1), _key(1, 1, 0), _key(0, 0, -1)]
    k27 = full_search(G, 27)
    assert k27[2] == _key(1, 1, 1)  # (4/sqrt 3 > 3/sqrt 2)
