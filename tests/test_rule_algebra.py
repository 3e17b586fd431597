"""The word-level algebra the HIP kernels apply to 32 sites at a time, checked
bit by bit on the CPU over every neighbourhood: the T = 0 rule (Methods,
equ:glauberAcceptance: flip when the energy falls, and with a fair tie bit
when it stays equal) written as a majority of seven, its tie test, and the
two forms of the fused bond count (sum over one colour of the anti-aligned
neighbour count a).  The kernels themselves are checked against the oracle
on the GPU; this pins the identities their code relies on."""
import itertools


def maj(a, b, c):
    return int(a + b + c >= 2)


def plain_rule(s, nbrs, r):
    """New spin (1 = up) by the definition: a = anti-aligned neighbours; flip
    iff a >= 4, or a == 3 and r == 1."""
    a = sum(1 for v in nbrs if v != s)
    return 1 - s if (a >= 4 or (a == 3 and r == 1)) else s


def cases():
    for bits in itertools.product((0, 1), repeat=8):
        yield bits[0], bits[1:7], bits[7]


def triples(n):
    xa, ma = n[0] ^ n[1] ^ n[2], maj(n[0], n[1], n[2])
    xb, mb = n[3] ^ n[4] ^ n[5], maj(n[3], n[4], n[5])
    return xa, ma, xb, mb


def test_majority_of_seven_is_the_rule():
    for s, n, r in cases():
        xa, ma, xb, mb = triples(n)
        assert maj(ma, mb, maj(xa, xb, s ^ r)) == plain_rule(s, n, r), (s, n, r)


def test_tie_test():
    for s, n, r in cases():
        xa, ma, xb, mb = triples(n)
        a = sum(1 for v in n if v != s)
        assert ((xa ^ xb) & (ma ^ mb)) == int(a == 3), (s, n)


def test_split_form_base_and_tie():
    # new = base ^ (tie & r): base = the rule with r = 0
    for s, n, r in cases():
        xa, ma, xb, mb = triples(n)
        tie = (xa ^ xb) & (ma ^ mb)
        base = maj(ma, mb, maj(xa, xb, s))
        assert base ^ (tie & r) == plain_rule(s, n, r)


def test_bond_count_from_the_triples():
    for s, n, _ in cases():
        xa, ma, xb, mb = triples(n)
        a = sum(1 for v in n if v != s)
        assert a == (xa ^ s) + (xb ^ s) + 2 * ((ma ^ s) + (mb ^ s)), (s, n)


def test_bit_sliced_antialigned_count():
    # U = up neighbours as three bit planes (u2 u1 u0); a = U for a down
    # spin, 6 - U for an up one: a0 = u0, a1 = u1 ^ (s & ~u0),
    # a2 = u2 ^ (s & ~(u1 & u0))
    for s, n, _ in cases():
        xa, ma, xb, mb = triples(n)
        k = xa & xb
        u0, u1, u2 = xa ^ xb, ma ^ mb ^ k, maj(ma, mb, k)
        assert 4 * u2 + 2 * u1 + u0 == sum(n)
        a1 = u1 ^ (s & (1 - u0))
        a2 = u2 ^ (s & (1 - (u1 & u0)))
        a = sum(1 for v in n if v != s)
        assert a == u0 + 2 * a1 + 4 * a2, (s, n)
