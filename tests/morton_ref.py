"""Morton (Z-order) permutation of the documented keys, in numpy: shared by
the GPU tests that check the reordering bit for bit and those that replay a
reordered evaluation on the oracle."""
import numpy as np


def morton_reference(x, y):
    """Permutation of the documented keys: 16-bit quantisation over the bounding
    box, x in the even bits, ties broken by the input index."""
    def q(v):
        lo, hi = v.min(), v.max()
        span = hi - lo
        if not span > 0:
            return np.zeros(v.size, dtype=np.uint64)
        f = np.floor((v - lo) / span * 65535.0)
        return np.clip(f, 0, 65535).astype(np.uint64)

    def spread(v):
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v
    code = spread(q(x)) | (spread(q(y)) << np.uint64(1))
    keys = (code << np.uint64(32)) | np.arange(x.size, dtype=np.uint64)
    return np.argsort(keys, kind="stable")
