"""Helpers shared by the GPU tests: bit-exact comparison of pair arrays."""
import numpy as np


def diff_pairs(a, b):
    """None when equal field by field (floats compared bitwise), else a message."""
    if len(a) != len(b):
        return "count %d != %d" % (len(a), len(b))
    for f in a.dtype.names:
        x, y = np.asarray(a[f]), np.asarray(b[f])
        if x.dtype == np.float32:
            x, y = x.view(np.uint32), y.view(np.uint32)
        bad = np.nonzero(x != y)[0]
        if len(bad):
            j = int(bad[0])
            return "field %s differs at %d: %r vs %r (first of %d)" % (f, j, a[j], b[j], len(bad))
    return None
