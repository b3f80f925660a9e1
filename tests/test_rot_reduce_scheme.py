"""The lane schedule of the select-free rotated reduction of the register kernels, checked on the host
by simulating which spectral index and which lanes' partial sums every register position holds.

Lane n2 (of G >= P lanes, P a power of two) holds its P spectral values shifted by s = bitrev(n2 mod P):
position p holds index (p + s) mod P. In step j every lane keeps positions [0, h), h = P >> (j + 1),
and adds positions [h, 2h) of lane n2 ^ x_j with x_0 = 1, x_1 = 2 or 3 (bit 1 of n2 set or not) and
x_j = 2^j | (bit j of n2 set ? 0 : x_(j-1)); the remaining lane bits are summed in full. Afterwards
every lane must hold the sum over all G lanes of index bitrev(n2 mod P), the value the cross-lane
inverse expects, and each step must add disjoint partial sums of equal indices. The same sets are
checked for the plain power-of-two DFT identity on random data.
"""

import numpy as np
import pytest


def bitrev(v, bits):
    r = 0
    for b in range(bits):
        r |= ((v >> b) & 1) << (bits - 1 - b)
    return r


def partner_mask(n2, j):
    x = 1
    for jj in range(1, j + 1):
        if jj == 1:
            x = 2 if (n2 >> 1) & 1 else 3
        else:
            x = (1 << jj) | (0 if (n2 >> jj) & 1 else x)
    return x


@pytest.mark.parametrize("P,G", [(2, 2), (2, 8), (4, 4), (4, 8), (8, 8), (8, 32), (16, 16), (16, 32), (32, 64)])
def test_rotated_reduction_sums_every_lane_into_bitrev_index(P, G):
    L = P.bit_length() - 1
    s = [bitrev(n % P, L) for n in range(G)]
    held = [[((p + s[n]) % P, frozenset([n])) for p in range(P)] for n in range(G)]
    for j in range(L):
        h = P >> (j + 1)
        new = []
        for n in range(G):
            m = n ^ partner_mask(n, j)
            assert 0 <= m < G and (m // P) == (n // P)  # the partner stays in the lane's group of P
            keep, recv = held[n][:h], held[m][h:2 * h]
            for (ka, la), (kb, lb) in zip(keep, recv):
                assert ka == kb and not (la & lb)
            new.append([(ka, la | lb) for (ka, la), (kb, lb) in zip(keep, recv)])
        held = new
    for bit in range(L, G.bit_length() - 1):  # lane bits above log2 P: all-reduce
        held = [[(k, a | held[n ^ (1 << bit)][0][1])] for n, [(k, a)] in enumerate(held)]
    for n in range(G):
        (k, lanes), = held[n]
        assert k == bitrev(n % P, L)
        assert lanes == frozenset(range(G))


@pytest.mark.parametrize("P,G", [(4, 8), (8, 8), (8, 16)])
def test_rotated_reduction_on_data(P, G):
    # numeric check: lane spectra V[n2] (with the shift applied by modulating the input) reduced by
    # the schedule give sum_n2 V[n2][bitrev(n2 mod P)] in lane n2
    rng = np.random.default_rng(7)
    L = P.bit_length() - 1
    x = rng.standard_normal((G, P)) + 1j * rng.standard_normal((G, P))
    n1 = np.arange(P)
    vals = []
    for n in range(G):
        sh = bitrev(n % P, L)
        vals.append(np.fft.fft(x[n] * np.exp(-2j * np.pi * sh * n1 / P)))  # position p holds index p + sh
    for j in range(L):
        h = P >> (j + 1)
        vals = [vals[n][:h] + vals[n ^ partner_mask(n, j)][h:2 * h] for n in range(G)]
    for bit in range(L, G.bit_length() - 1):
        vals = [vals[n] + vals[n ^ (1 << bit)] for n in range(G)]
    full = np.fft.fft(x, axis=1).sum(axis=0)
    for n in range(G):
        assert abs(vals[n][0] - full[bitrev(n % P, L)]) <= 1e-12 * np.abs(full).max()
