"""The SPAI parameter layout agrees between the library, its trainer and the oracle (CPU)."""
import numpy as np

from oracle import spai_oracle as SO


def test_layout_agrees():
    import paper_1710_07080_amd as P
    from paper_1710_07080_amd import spai_train as T

    assert P.isira.spai_nparam() == SO.NPARAM == T.NPARAM == 1010
    for name, (o, sz) in SO.OFF.items():
        assert T.OFFSETS[name][:2] == (o, sz), name


def test_committed_weights_are_well_formed():
    import os

    from paper_1710_07080_amd import spai_train as T

    if not os.path.exists(T.DEFAULT_WEIGHTS):
        return
    a = np.load(T.DEFAULT_WEIGHTS, allow_pickle=False)
    assert a.dtype == np.float32 and a.shape == (T.NPARAM,)
    assert np.all(np.isfinite(a))
