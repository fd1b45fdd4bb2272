"""Host-side input checks of the Python binding: a malformed coordinate or
triangle array is refused before anything reaches the library."""
import numpy as np
import pytest

import paper_2403_14723_amd as gp


@pytest.mark.parametrize("shape,cols", [((5, 4), 3), ((7,), 3), ((3, 3, 3), 3), ((4, 3), 2), ((9,), 2)])
def test_malformed_host_inputs_raise(shape, cols):
    a = np.zeros(shape, dtype=np.int32)
    with pytest.raises(ValueError):
        gp._as_input(a, cols)


@pytest.mark.parametrize("shape,cols,n", [((5, 3), 3, 5), ((12,), 3, 4), ((6, 2), 2, 6), ((0, 3), 3, 0)])
def test_wellformed_host_inputs(shape, cols, n):
    a = np.arange(int(np.prod(shape)), dtype=np.int64).reshape(shape)
    ptr, cnt, keep, dev = gp._as_input(a, cols)
    assert cnt == n and not dev
    assert keep.dtype == np.int32 and keep.shape == (n, cols)
    assert np.array_equal(keep.ravel(), a.ravel().astype(np.int32))
