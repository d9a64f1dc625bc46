"""Philox4x32-10 and the Box-Muller normals of the synthetic-noise stream,
written out in numpy (test infrastructure: the reference the device noise is
checked against). Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011."""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: uint64 array [..., 4] of 32-bit words; key: (k0, k1). Returns the
    four output words (uint64 array [..., 4])."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    for _ in range(10):
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return np.stack(c, axis=-1)


def normals(n, seed):
    """The first n variates of the stream `seed` (FP64)."""
    g = np.arange((n + 3) // 4, dtype=np.uint64)
    ctr = np.stack([g & np.uint64(MASK), g >> np.uint64(32), np.zeros_like(g), np.zeros_like(g)],
                   axis=-1)
    w = philox4x32_10(ctr, (seed & MASK, (seed >> 32) & MASK)).astype(np.float64)
    u = (np.floor(w / 256.0) + 0.5) * 2.0 ** -24
    ra = np.sqrt(-2.0 * np.log(u[:, 0]))
    rb = np.sqrt(-2.0 * np.log(u[:, 2]))
    out = np.stack([ra * np.cos(2 * np.pi * u[:, 1]), ra * np.sin(2 * np.pi * u[:, 1]),
                    rb * np.cos(2 * np.pi * u[:, 3]), rb * np.sin(2 * np.pi * u[:, 3])], axis=-1)
    return out.reshape(-1)[:n]
