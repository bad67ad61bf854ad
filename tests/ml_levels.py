"""Test helper: the oracle's multilevel hierarchy with the library's level matrices in place
of its own (the same aggregates; the entries differ only in rounding, which
test_multilevel_shape.py pins entry by entry).  The oracle's cycle over these matrices is the
reference for the GPU cycle without the coarsest solve's amplification of those roundings."""
import copy

import numpy as np
import scipy.sparse as sp


def hierarchy_with_library_matrices(P, g, trim, h, coarse_max):
    hl = copy.copy(h)
    hl.A = []
    pi = np.delete(np.arange(g.n), trim)  # oracle vertex -> library vertex on this level
    for lvl, A in enumerate(h.A):
        W, dg, agg = P.isira.ml_level_matrix(g, trim, lvl, coarse_max=coarse_max)
        hl.A.append((sp.diags(dg) - W).tocsr()[pi][:, pi].tocsr())
        if lvl + 1 < len(h.A):
            agg_o = h.agg[lvl]
            nxt = -np.ones(h.A[lvl + 1].shape[0], dtype=np.int64)
            mem = np.flatnonzero(agg_o >= 0)
            nxt[agg_o[mem]] = agg[pi[mem]]
            pi = nxt
    return hl
