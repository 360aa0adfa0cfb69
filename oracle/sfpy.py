"""Second, pure-Python transcription of SF_F -- TEST INFRASTRUCTURE ONLY.

Written separately from the C oracle (different language, different hash
implementation: scikit-learn's MurmurHash3_x86_32) so the two can check each
other on tiny streams.  Lists of Python ints, no numpy arithmetic.

Notation follows the paper (Section 3.4/3.5): Slim A[i][j], Fat B[i][j][k],
bucket hash h_i, slot hash f_i, B_e^min.  Slim counters saturate at 65535.
"""
from __future__ import annotations

from sklearn.utils import murmurhash3_32

SLIM_MAX = 65535


def row_hash(key, seed: int) -> int:
    """MurmurHash3_x86_32 of the key's bytes (uint32 keys: 4 little-endian bytes)."""
    if isinstance(key, (bytes, bytearray)):
        return murmurhash3_32(bytes(key), seed=seed, positive=True)
    return murmurhash3_32(int(key).to_bytes(4, "little"), seed=seed, positive=True)


class SF:
    def __init__(self, d: int, w: int, z: int, seed_base: int = 1):
        self.d, self.w, self.z, self.seed_base = d, w, z, seed_base
        self.A = [[0] * w for _ in range(d)]
        self.B = [[[0] * z for _ in range(w)] for _ in range(d)]

    def idx(self, key):
        """Eq. (1) with 0-based indices: c = g mod wz, h = c mod w, f = c div w."""
        out = []
        for i in range(self.d):
            c = row_hash(key, self.seed_base + i) % (self.w * self.z)
            out.append((c % self.w, c // self.w))
        return out

    # ---- sequential SF_F
    def insert_at(self, hf):
        for i, (h, f) in enumerate(hf):
            self.B[i][h][f] += 1
        b_min = min(self.B[i][h][f] for i, (h, f) in enumerate(hf))
        a_vals = [self.A[i][h] for i, (h, _) in enumerate(hf)]
        m = min(a_vals)
        if m < b_min and m < SLIM_MAX:
            for i, (h, _) in enumerate(hf):
                if self.A[i][h] == m:
                    self.A[i][h] = m + 1

    def delete_at(self, hf):
        for i, (h, f) in enumerate(hf):
            old_max = max(self.B[i][h])
            self.B[i][h][f] -= 1
            new_max = max(self.B[i][h])
            if new_max != old_max and self.A[i][h] > new_max:
                self.A[i][h] = new_max

    def query_at(self, hf) -> int:
        return min(self.A[i][h] for i, (h, _) in enumerate(hf))

    def seq(self, stream):
        """stream: iterable of (key, is_delete)."""
        for key, dele in stream:
            (self.delete_at if dele else self.insert_at)(self.idx(key))

    # ---- deterministic batch schedule (same definition as the C oracle's batch(b))
    def batch(self, stream, b: int):
        stream = list(stream)
        for lo in range(0, len(stream), b):
            part = [(self.idx(k), dele) for k, dele in stream[lo:lo + b]]
            ins = [hf for hf, dele in part if not dele]
            dels = [hf for hf, dele in part if dele]
            snap = []
            for hf in ins:                                       # S1
                m0 = min(self.A[i][h] for i, (h, _) in enumerate(hf))
                pre = [self.B[i][h][f] for i, (h, f) in enumerate(hf)]
                snap.append((m0, pre))
            for hf in ins:                                       # S2
                for i, (h, f) in enumerate(hf):
                    self.B[i][h][f] += 1
            for hf, (m0, pre) in zip(ins, snap):                 # S3
                post = [self.B[i][h][f] for i, (h, f) in enumerate(hf)]
                t = min(m0 + min(p - q for p, q in zip(post, pre)), max(m0, min(post)), SLIM_MAX)
                for i, (h, _) in enumerate(hf):
                    self.A[i][h] = max(self.A[i][h], t)
            for hf in dels:                                      # S4
                for i, (h, f) in enumerate(hf):
                    self.B[i][h][f] -= 1
            for hf in dels:                                      # S5
                for i, (h, _) in enumerate(hf):
                    self.A[i][h] = min(self.A[i][h], max(self.B[i][h]))

    def query(self, key) -> int:
        return self.query_at(self.idx(key))
