"""The no-allocation Gram product against the workspace form.

mbbs_gram_noalloc keeps its partial sums in a static device buffer instead
of a caller workspace; it runs the same kernels in the same order, so its
result must equal mbbs_gram's bit for bit.  Two calls in a row, the second
with a smaller input (fewer rows and a narrower block), check that the
buffer's contents from the first call do not leak into the second.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
torch = gu.torch
B = gu.binding


def _pair(N, L, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, L)) + 1j * rng.standard_normal((N, L))
    Y = rng.standard_normal((N, L)) + 1j * rng.standard_normal((N, L))
    return X, Y


def _both(N, L, seed):
    X, Y = _pair(N, L, seed)
    Xd, Yd = gu.dev(X), gu.dev(Y)
    ws = torch.empty(B.mbbs_gram_workspace_size(N, L), dtype=torch.uint8, device="cuda")
    G1 = torch.empty((L, L), dtype=torch.complex128, device="cuda")
    G2 = torch.empty((L, L), dtype=torch.complex128, device="cuda")
    B.mbbs_gram(N, L, Xd, Yd, G1, ws)
    B.mbbs_gram_noalloc(N, L, Xd, Yd, G2)
    return X, Y, gu.host(G1), gu.host(G2)


def test_noalloc_gram_equals_workspace_form_twice():
    gu.flush("no-alloc Gram: large then small")
    for N, L, seed in ((12 * 65536 + 37, 12, 1), (12 * 777, 5, 2)):
        X, Y, g_ws, g_na = _both(N, L, seed)
        assert g_na.tobytes() == g_ws.tobytes(), (N, L)
        ref = X.conj().T @ Y
        np.testing.assert_allclose(g_na, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_noalloc_gram_rejects_sizes_beyond_the_scratch():
    X, Y = _pair(64, 2, 3)
    Xd, Yd = gu.dev(X), gu.dev(Y)
    G = torch.empty((17, 17), dtype=torch.complex128, device="cuda")
    for L in (0, 17):
        with pytest.raises(B.MbbsError) as e:
            B.mbbs_gram_noalloc(64, L, Xd, Yd, G)
        assert e.value.code == B.EINVAL
