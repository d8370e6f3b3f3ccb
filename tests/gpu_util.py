"""Helpers shared by the GPU tests: bit-exact comparison of pair arrays, and the device the
GPU tests run on."""
import os

import numpy as np

HOST_LIBRARY_ENV = "FC_TEST_HOST_LIBRARY"


def device_for_tests(fc, torch):
    """(device, host_mode) for the GPU test modules.

    On a GPU: cuda:0.  Without one, if FC_TEST_HOST_LIBRARY names the host build of the C ABI
    (tests/cpu_emulation, variant "so"), the GPU tests run against it on host tensors, which
    checks the tests themselves; otherwise (None, False) and the module skips."""
    if torch.cuda.is_available():
        return torch.device("cuda:0"), False
    so = os.environ.get(HOST_LIBRARY_ENV)
    if so:
        fc.LIB_PATH = so
        return torch.device("cpu"), True
    return None, False


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
