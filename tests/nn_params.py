"""Parameter-vector layout of the learned model (W0, b0, ..., W4, b4, then the
hash table) and a seeded random parameter generator for tests."""
import math

import numpy as np

FIN = [35, 64, 64, 64, 64]
FOUT = [64, 64, 64, 64, 256]


def layout(n_params):
    """Offsets and sizes of W0,b0,...,W4,b4 and of the table."""
    off, segs = 0, {}
    for k in range(5):
        segs["W%d" % k] = (off, FOUT[k] * FIN[k])
        off += FOUT[k] * FIN[k]
        segs["b%d" % k] = (off, FOUT[k])
        off += FOUT[k]
    segs["table"] = (off, n_params - off)
    return segs


def random_params(n_params, rng, scale=0.3, table_scale=0.5):
    lay = layout(n_params)
    p = np.zeros(n_params, np.float32)
    for k in range(5):
        a, m = lay["W%d" % k]
        p[a:a + m] = rng.normal(0, scale * math.sqrt(2.0 / FIN[k]), m)
        a, m = lay["b%d" % k]
        p[a:a + m] = rng.normal(0, 0.1, m)
    a, m = lay["table"]
    p[a:a + m] = rng.normal(0, table_scale, m)
    return p
