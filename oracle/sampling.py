"""Oracle of the seeded MPPI perturbations (Sec. IV-A sampling).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this module; the library has its own generator and shares
nothing with this one.

The perturbation of rollout k at step n of MPPI iteration i is sigma * z,
z standard normal, from the counter-based generator Philox4x64-10 (Salmon,
Moraes, Dror and Shaw, SC 2011) keyed by (seed, 0) at counter
(n // 4, k, i, 0), followed by the Box-Muller transform (Box and Muller
1958). Written from those definitions in plain Python integers, one block at
a time: no vectorisation, no shared tables.

Pins (tests/test_sampling.py): the block function against numpy's own
Philox (its raw 64-bit output at a given counter and key), the uniforms'
range, and the normals' moments and distribution.
"""
import math

MASK64 = (1 << 64) - 1
# round multipliers and key increments of Philox4x64 (Salmon et al., Table 2)
M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: four 64-bit words from a 4-word counter and a
    2-word key."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & MASK64, (k1 + W1) & MASK64
        p0 = M0 * c0      # exact 128-bit products
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64, (p0 >> 64) ^ c3 ^ k1,
                          p0 & MASK64)
    return [c0, c1, c2, c3]


def uniform_open0(w):
    """53-bit uniform in (0, 1] from the top bits of a 64-bit word."""
    return ((w >> 11) + 1) * 2.0 ** -53


def uniform_open1(w):
    """53-bit uniform in [0, 1) from the top bits of a 64-bit word."""
    return (w >> 11) * 2.0 ** -53


def box_muller(wa, wb):
    """Two standard normals from two 64-bit words."""
    r = math.sqrt(-2.0 * math.log(uniform_open0(wa)))
    t = 6.283185307179586 * uniform_open1(wb)
    return r * math.cos(t), r * math.sin(t)


def eps(seed, iteration, K, H, sigma):
    """Perturbations [K][H] (lists of floats) of one MPPI iteration."""
    out = []
    for k in range(K):
        row = []
        for n in range(H):
            j, q = divmod(n, 4)
            w = philox4x64_10((j, k, iteration, 0), (seed, 0))
            z = box_muller(w[2 * (q // 2)], w[2 * (q // 2) + 1])[q % 2]
            row.append(sigma * z)
        out.append(row)
    return out
