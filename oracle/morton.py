"""Oracle for Morton keys and oct-neighbour search (plain Python/NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Morton key (section "Morton key encoding and neighbour arithmetic", equation
  morton_encode; appendix "Morton key encoding details", algorithm "Morton key
  encoding"): bit b of x goes to key bit 3b, of y to 3b+1, of z to 3b+2, with
  B = 21 bits per coordinate for a 64-bit key.  Written here as the bit loop
  over b, the slow and obviously correct form.
* neighbour key (algorithm "Morton neighbour key in direction j"): decode,
  step one coordinate by +-1, wrap periodically modulo the level's extent,
  re-encode.
* parent and child keys: M >> 3 and (M << 3) | child.
* neighbour search by brute force: the oct whose integer coordinates equal
  this oct's plus the unit step (periodic), found by direct comparison; -1
  when no such oct exists.
* 128-bit keys (same section: B = 42 bits per coordinate, key bits 0..125):
  the same bit loop on Python integers; as arrays they are [n, 2] uint64
  words, low word first.
* the per-level key -> grid-index table (appendix "Per-level hash table and
  replacement functions": insert when a grid is made, delete when it is
  killed, look up): its observable behaviour is that of a map, written here
  as a Python dict (:class:`KeyMap`).  Slot placement, probing and rehashing
  are not observable through lookups and are not modelled.
* the table's hash (same appendix, equation hash_func): the key is first
  reduced to 64 bits (a 64-bit key as it is, a 128-bit key by XOR of its two
  halves), then t = ((h * phi1) XOR (h >> 16)) * phi2 and
  h(M) = t XOR (t >> 13), with products taken modulo 2^64 and logical shifts;
  the home slot is h(M) modulo the power-of-two capacity.  Evaluated here on
  Python integers (:func:`table_hash`).

Directions are numbered j = 0..5 as -x, +x, -y, +y, -z, +z.
"""
from __future__ import annotations

import numpy as np

B64 = 21
B128 = 42
DIRS = np.array([(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)], dtype=np.int64)

__all__ = ["B64", "B128", "DIRS", "encode", "decode", "encode_array", "encode_array128", "words_to_int",
           "neighbour_key", "parent_key", "child_key", "neighbours_bruteforce", "neighbours_sorted", "KeyMap",
           "HASH_PHI1", "HASH_PHI2", "table_hash", "home_slot"]

# the two multipliers of equation hash_func
HASH_PHI1 = 2654435761
HASH_PHI2 = 0x9E3779B97F4A7C15
_MASK64 = (1 << 64) - 1


def encode(ix: int, iy: int, iz: int, bits: int = B64) -> int:
    """Interleave the bits of (ix, iy, iz): the bit loop of the encoding algorithm."""
    m = 0
    for b in range(bits):
        m |= ((ix >> b) & 1) << (3 * b)
        m |= ((iy >> b) & 1) << (3 * b + 1)
        m |= ((iz >> b) & 1) << (3 * b + 2)
    return m


def decode(m: int, bits: int = B64) -> tuple[int, int, int]:
    """Inverse of :func:`encode`."""
    ix = iy = iz = 0
    for b in range(bits):
        ix |= ((m >> (3 * b)) & 1) << b
        iy |= ((m >> (3 * b + 1)) & 1) << b
        iz |= ((m >> (3 * b + 2)) & 1) << b
    return ix, iy, iz


def encode_array(ijk: np.ndarray, bits: int = B64) -> np.ndarray:
    """Vectorised bit loop over an [n, 3] array of coordinates -> uint64 keys."""
    ijk = np.asarray(ijk, dtype=np.uint64)
    m = np.zeros(len(ijk), dtype=np.uint64)
    one = np.uint64(1)
    for b in range(bits):
        bb = np.uint64(b)
        for d in range(3):
            m |= ((ijk[:, d] >> bb) & one) << np.uint64(3 * b + d)
    return m


def encode_array128(ijk: np.ndarray) -> np.ndarray:
    """Vectorised bit loop with B = 42 -> [n, 2] uint64 (low word, high word)."""
    ijk = np.asarray(ijk, dtype=np.uint64)
    out = np.zeros((len(ijk), 2), dtype=np.uint64)
    one = np.uint64(1)
    for b in range(B128):
        for d in range(3):
            pos = 3 * b + d
            out[:, pos >> 6] |= ((ijk[:, d] >> np.uint64(b)) & one) << np.uint64(pos & 63)
    return out


def words_to_int(w) -> int:
    """[low, high] uint64 words -> the 128-bit key as a Python integer."""
    return int(w[0]) | (int(w[1]) << 64)


def neighbour_key(m: int, j: int, n_dim: int, bits: int = B64) -> int:
    """Key of the same-level neighbour in direction j, with periodic wrap at n_dim."""
    c = list(decode(m, bits))
    d = j // 2
    c[d] = (c[d] + (1 if j % 2 else -1)) % n_dim
    return encode(c[0], c[1], c[2], bits)


def parent_key(m: int) -> int:
    return m >> 3


def child_key(m: int, child: int) -> int:
    return (m << 3) | child


def neighbours_bruteforce(oct_ijk: np.ndarray, n_dim: int) -> np.ndarray:
    """[n_oct, 6] int32 neighbour oct indices by all-pairs comparison (small inputs)."""
    ijk = np.asarray(oct_ijk, dtype=np.int64)
    n = len(ijk)
    out = np.full((n, 6), -1, dtype=np.int32)
    for j in range(6):
        tgt = (ijk + DIRS[j]) % n_dim
        eq = np.all(tgt[:, None, :] == ijk[None, :, :], axis=2)      # [n, n]
        has = eq.any(axis=1)
        out[has, j] = np.argmax(eq[has], axis=1)
    return out


def neighbours_sorted(oct_ijk: np.ndarray, n_dim: int) -> np.ndarray:
    """Same result as :func:`neighbours_bruteforce` by sort + binary search (any size)."""
    ijk = np.asarray(oct_ijk, dtype=np.int64)

    def lin(c):
        return (c[:, 2] * n_dim + c[:, 1]) * n_dim + c[:, 0]

    keys = lin(ijk)
    order = np.argsort(keys)
    sk = keys[order]
    out = np.full((len(ijk), 6), -1, dtype=np.int32)
    for j in range(6):
        q = lin((ijk + DIRS[j]) % n_dim)
        pos = np.minimum(np.searchsorted(sk, q), len(sk) - 1)
        hit = sk[pos] == q
        out[hit, j] = order[pos[hit]]
    return out


class KeyMap:
    """The table's contract as a map from key to grid index (a dict).

    ``insert`` sets the value of each key (a key already present takes the new
    value; a key repeated inside one batch keeps one of its values, so callers
    compare such keys by membership only); ``erase`` removes the keys present;
    ``lookup`` gives the value or -1.
    """

    def __init__(self):
        self.d: dict[int, int] = {}

    def insert(self, keys, vals) -> None:
        for k, v in zip(keys, vals):
            self.d[int(k)] = int(v)

    def erase(self, keys) -> int:
        n = 0
        for k in keys:
            if self.d.pop(int(k), None) is not None:
                n += 1
        return n

    def lookup(self, keys) -> np.ndarray:
        return np.array([self.d.get(int(k), -1) for k in keys], dtype=np.int32)

    def __len__(self) -> int:
        return len(self.d)


def table_hash(key: int, key_words: int = 1) -> int:
    """Equation hash_func of a Morton key (Python integers, unsigned 64-bit).

    ``key_words`` = 2: a 128-bit key (a Python integer up to 2^128), reduced to
    64 bits by XOR of its upper and lower halves before hashing.
    """
    k = int(key)
    if key_words == 2:
        h = (k & _MASK64) ^ (k >> 64)
    else:
        h = k & _MASK64
    t = (((h * HASH_PHI1) & _MASK64) ^ (h >> 16)) * HASH_PHI2 & _MASK64
    return t ^ (t >> 13)


def home_slot(key: int, capacity: int, key_words: int = 1) -> int:
    """First probed slot of a key in a table of ``capacity`` (a power of two) slots."""
    return table_hash(key, key_words) & (capacity - 1)
