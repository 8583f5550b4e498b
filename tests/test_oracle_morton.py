"""Pins for the Morton-key and neighbour oracle: hand-derived keys, round
trips, parent/child identities, periodic wrap and two independent searches
(the paper's own unit-test list for its key module, for 64-bit keys and for
128-bit keys across the word boundary), and the key map against a list scan."""
import numpy as np

from oracle import morton as M


def test_hand_derived_keys():
    assert M.encode(0, 0, 0) == 0
    assert M.encode(1, 0, 0) == 1
    assert M.encode(0, 1, 0) == 2
    assert M.encode(0, 0, 1) == 4
    assert M.encode(1, 1, 1) == 7
    assert M.encode(2, 0, 0) == 8
    assert M.encode(3, 3, 3) == 63
    assert M.encode(5, 0, 0) == 0b001000001        # bits 0 and 2 of x -> key bits 0 and 6
    assert M.encode(0, 0, 1 << 20) == 1 << 62       # top bit of z -> bit 62, bit 63 unused
    top = (1 << 21) - 1
    assert M.encode(top, top, top) == (1 << 63) - 1


def test_octant_order_matches_child_index():
    # inside a 2x2x2 block the key is cx + 2cy + 4cz, the oct-major cell index
    for c in range(8):
        assert M.encode(c & 1, (c >> 1) & 1, (c >> 2) & 1) == c


def test_round_trip_all_small_and_random():
    for x in range(0, 128, 7):
        for y in range(0, 128, 5):
            for z in range(0, 128, 3):
                assert M.decode(M.encode(x, y, z)) == (x, y, z)
    rng = np.random.default_rng(0)
    ijk = rng.integers(0, 1 << 21, size=(2000, 3))
    keys = M.encode_array(ijk)
    for (x, y, z), k in zip(ijk[:300], keys[:300]):
        assert int(k) == M.encode(int(x), int(y), int(z))
        assert M.decode(int(k)) == (x, y, z)
    assert len(np.unique(keys)) == len(np.unique(ijk, axis=0))


def test_parent_child_identities():
    rng = np.random.default_rng(1)
    for _ in range(200):
        x, y, z = (int(v) for v in rng.integers(0, 1 << 20, 3))
        m = M.encode(x, y, z)
        for c in range(8):
            ch = M.child_key(m, c)
            assert M.parent_key(ch) == m
            assert M.decode(ch) == (2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2))
        assert M.decode(M.parent_key(m)) == (x >> 1, y >> 1, z >> 1)


def test_neighbour_walk_wraps():
    n = 8
    m = M.encode(n - 1, 0, 3)
    assert M.decode(M.neighbour_key(m, 1, n)) == (0, 0, 3)       # +x wraps
    assert M.decode(M.neighbour_key(m, 2, n)) == (n - 1, n - 1, 3)  # -y wraps
    assert M.decode(M.neighbour_key(m, 5, n)) == (n - 1, 0, 4)
    # a full walk of n steps returns to the start
    k = m
    for _ in range(n):
        k = M.neighbour_key(k, 4, n)
    assert k == m


def test_bruteforce_equals_sorted_search():
    rng = np.random.default_rng(2)
    n = 16
    allc = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    sel = allc[rng.random(len(allc)) < 0.3]
    sel = sel[rng.permutation(len(sel))][:900]
    a = M.neighbours_bruteforce(sel, n)
    b = M.neighbours_sorted(sel, n)
    np.testing.assert_array_equal(a, b)
    # every found neighbour really is at the unit step; absent ones really are absent
    s = set(map(tuple, sel))
    for j in range(6):
        for i in range(0, len(sel), 37):
            t = tuple((sel[i] + M.DIRS[j]) % n)
            if a[i, j] >= 0:
                assert tuple(sel[a[i, j]]) == t
            else:
                assert t not in s


def test_hand_derived_keys_128():
    # bit b of x, y, z -> key bits 3b, 3b+1, 3b+2: bit 21 of x lands on key
    # bit 63, of y on 64 and of z on 65 (the first bits of the high word)
    assert M.encode(1 << 21, 0, 0, M.B128) == 1 << 63
    assert M.encode(0, 1 << 21, 0, M.B128) == 1 << 64
    assert M.encode(0, 0, 1 << 21, M.B128) == 1 << 65
    assert M.encode(0, 0, 1 << 41, M.B128) == 1 << 125
    top = (1 << 42) - 1
    assert M.encode(top, top, top, M.B128) == (1 << 126) - 1
    # 64-bit keys are the 128-bit keys of coordinates below 2^21
    assert M.encode(123, 456, 789, M.B128) == M.encode(123, 456, 789)
    w = M.encode_array128(np.array([[1 << 21, 0, 0], [0, 1 << 21, 0], [top, top, top], [5, 0, 0]]))
    assert [M.words_to_int(r) for r in w] == [1 << 63, 1 << 64, (1 << 126) - 1, 0b1000001]


def test_round_trip_and_relatives_128():
    rng = np.random.default_rng(3)
    ijk = rng.integers(0, 1 << 42, size=(400, 3), dtype=np.int64)
    ijk[:4] = [[(1 << 21) - 1, (1 << 21), (1 << 21) + 1], [1 << 41, 0, 1], [0, 0, 0], [(1 << 42) - 1] * 3]
    w = M.encode_array128(ijk)
    for (x, y, z), r in zip(ijk, w):
        k = M.words_to_int(r)
        assert k == M.encode(int(x), int(y), int(z), M.B128)
        assert M.decode(k, M.B128) == (x, y, z)
        assert M.decode(M.parent_key(k), M.B128) == (x >> 1, y >> 1, z >> 1)
        if x < (1 << 41) and y < (1 << 41) and z < (1 << 41):
            for c in (0, 5, 7):
                ch = M.child_key(k, c)
                assert M.decode(ch, M.B128) == (2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2))
                assert M.parent_key(ch) == k


def test_neighbour_walk_128_wraps_at_level_extent():
    n = 1 << 42                                   # level 43 with one root cell: the deepest
    m = M.encode(n - 1, (1 << 21) - 1, 0, M.B128)
    assert M.decode(M.neighbour_key(m, 1, n, M.B128), M.B128) == (0, (1 << 21) - 1, 0)
    assert M.decode(M.neighbour_key(m, 3, n, M.B128), M.B128) == (n - 1, 1 << 21, 0)   # crosses the word boundary
    assert M.decode(M.neighbour_key(m, 4, n, M.B128), M.B128) == (n - 1, (1 << 21) - 1, n - 1)


def test_keymap_against_list_scan():
    # the dict model against a list of (key, value) pairs scanned linearly
    rng = np.random.default_rng(4)
    km = M.KeyMap()
    pairs: list[list[int]] = []
    universe = [int(k) for k in rng.integers(0, 1 << 62, size=60)] + [(1 << 100) + 3, 1 << 64]
    for step in range(40):
        ks = [universe[i] for i in rng.choice(len(universe), size=8, replace=False)]
        if step % 3 == 2:
            km.erase(ks)
            pairs = [p for p in pairs if p[0] not in ks]
        else:
            vs = [int(v) for v in rng.integers(0, 1000, size=8)]
            km.insert(ks, vs)
            for k, v in zip(ks, vs):
                hit = [p for p in pairs if p[0] == k]
                if hit:
                    hit[0][1] = v
                else:
                    pairs.append([k, v])
        q = universe
        want = [next((p[1] for p in pairs if p[0] == k), -1) for k in q]
        assert km.lookup(q).tolist() == want
        assert len(km) == len(pairs)


# --- the table hash (appendix "Per-level hash table and replacement functions",
# equation hash_func; multipliers phi1 = 2654435761, phi2 = 0x9E3779B97F4A7C15
# as printed there) ---------------------------------------------------------
def _bits(v: int) -> str:
    """64-character binary string, most significant bit first."""
    return format(v, "064b")


def _shr(s: str, k: int) -> str:
    """Logical right shift of a 64-bit string: zeros enter at the top."""
    return ("0" * k + s)[:64]


def _xor(a: str, b: str) -> str:
    return "".join("1" if x != y else "0" for x, y in zip(a, b))


def _mul_mod64(a: int, b: int) -> int:
    """a * b mod 2^64 by schoolbook multiplication of 16-bit limbs."""
    la = [(a >> (16 * i)) & 0xFFFF for i in range(4)]
    lb = [(b >> (16 * i)) & 0xFFFF for i in range(4)]
    out = [0] * 4
    for i in range(4):
        carry = 0
        for j in range(4 - i):
            cur = out[i + j] + la[i] * lb[j] + carry
            out[i + j] = cur & 0xFFFF
            carry = cur >> 16
    return sum(v << (16 * i) for i, v in enumerate(out))


def _hash_by_limbs(h: int) -> int:
    phi1, phi2 = 2654435761, 0x9E3779B97F4A7C15
    t = _mul_mod64(int(_xor(_bits(_mul_mod64(h, phi1)), _shr(_bits(h), 16)), 2), phi2)
    return int(_xor(_bits(t), _shr(_bits(t), 13)), 2)


def test_table_hash_against_limb_arithmetic():
    assert M.HASH_PHI1 == 2654435761 and M.HASH_PHI2 == 0x9E3779B97F4A7C15
    assert M.table_hash(0) == 0
    rng = np.random.default_rng(11)
    keys = [1, 2, 7, 1 << 16, (1 << 16) + 1, (1 << 63) - 1, 1 << 63, (1 << 64) - 2, 0xFFFF0000FFFF0000]
    keys += [int(k) for k in rng.integers(0, 1 << 63, size=300, dtype=np.uint64)]
    keys += [M.encode(int(a), int(b), int(c)) for a, b, c in rng.integers(0, 1 << 21, size=(100, 3))]
    for k in keys:
        assert M.table_hash(k) == _hash_by_limbs(k), hex(k)
        assert 0 <= M.table_hash(k) < (1 << 64)


def test_table_hash_small_keys_invert_to_the_product():
    # keys below 2^16 have h >> 16 = 0, so t = k phi1 phi2 mod 2^64; undoing the
    # final xor-shift (t = h ^ (h >> 13) ^ (h >> 26) ^ ...) and multiplying by
    # the inverse of phi2 modulo 2^64 must give k phi1 mod 2^64
    inv2 = pow(0x9E3779B97F4A7C15, -1, 1 << 64)
    for k in (1, 3, 255, 4096, 65535):
        hk = M.table_hash(k)
        t, s = 0, hk
        while s:
            t ^= s
            s >>= 13
        assert (t * inv2) % (1 << 64) == (k * 2654435761) % (1 << 64)


def test_table_hash_128_folds_the_halves_and_home_slot_masks():
    rng = np.random.default_rng(12)
    for _ in range(50):
        lo, hi = (int(v) for v in rng.integers(0, 1 << 62, size=2, dtype=np.uint64))
        k = lo | (hi << 64)
        assert M.table_hash(k, key_words=2) == _hash_by_limbs(lo ^ hi)
        for cap in (16, 1 << 20):
            assert M.home_slot(k, cap, key_words=2) == _hash_by_limbs(lo ^ hi) % cap
    # a 64-bit key is the 128-bit key with a zero high word
    assert M.table_hash(12345, key_words=2) == M.table_hash(12345)
