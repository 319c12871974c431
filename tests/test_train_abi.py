"""Host-side checks of the training entry points (no GPU): argument validation and errors."""
import ctypes as C

import numpy as np
import pytest


@pytest.fixture(scope="module")
def L():
    from paper_2504_21627_amd import lsnif
    try:
        lsnif.load()
    except RuntimeError as e:
        pytest.skip(str(e))
    return lsnif


def test_trainer_needs_a_device_context(L):
    ctx = L.lsnif_create(-1)   # host-only
    try:
        with pytest.raises(L.LsnifError) as e:
            L.lsnif_trainer_create(ctx, 1)
        assert e.value.status == L.LSNIF_E_DEVICE
    finally:
        L.lsnif_destroy(ctx)


def test_null_arguments_are_errors(L):
    lib = L.load()
    out = C.c_void_p()
    assert lib.lsnif_trainer_create(None, 1, None, C.byref(out)) == L.LSNIF_E_INVALID
    assert lib.lsnif_train_grads(None, None, None, 0, None, None) == L.LSNIF_E_INVALID
    assert lib.lsnif_train_step(None, None, None, 0, None, None) == L.LSNIF_E_INVALID
    assert lib.lsnif_train_apply(None, None) == L.LSNIF_E_INVALID
    assert lib.lsnif_trainer_read(None, None, None, None, None, None) == L.LSNIF_E_INVALID
    lib.lsnif_trainer_destroy(None)   # a no-op


def test_target_record_layout(L):
    """lsnif_train_target is 36 bytes: hit, t, n[3], albedo[3], material."""
    assert L.TRAIN_TARGET.itemsize == 36
    t = L.targets_array([1, 0], [2.5, 9.0], [[0, 0, 1], [1, 0, 0]], [3, 1], [[0.1, 0.2, 0.3], [0, 0, 0]])
    assert t.shape == (2, 9) and t.dtype == np.float32
    rec = t.view(L.TRAIN_TARGET).ravel()
    assert rec["hit"].tolist() == [1, 0] and rec["material"].tolist() == [3, 1]
    assert rec["t"].tolist() == [2.5, 0.0]   # a miss's t is not read; stored as 0
    assert np.array_equal(rec["n"][0], [0, 0, 1]) and np.allclose(rec["albedo"][0], [0.1, 0.2, 0.3])
