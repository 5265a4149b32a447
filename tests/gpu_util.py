"""Helpers shared by the GPU tests: device tensors and lattice handles."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1104_0737_amd import binding  # noqa: E402

PH_AP = ((1.0, 0.0), (1.0, 0.0), (1.0, 0.0), (-1.0, 0.0))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_col_err(got, ref):
    got = got.reshape(-1, ref.shape[-1]) if got.ndim > 1 else got
    ref = ref.reshape(got.shape)
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


def max_elem_err(got, ref):
    """Per column: the largest elementwise deviation over the column's largest
    reference magnitude (a wrong value at a few sites, which a norm-wise
    comparison can hide, shows here)."""
    ref = ref.reshape(-1, ref.shape[-1])
    got = got.reshape(ref.shape)
    return np.max(np.abs(got - ref), axis=0) / np.max(np.abs(ref), axis=0)


class Lattice:
    def __init__(self, dims, block, U, kappa, phases=PH_AP):
        self.dims, self.block, self.kappa, self.phases = tuple(dims), tuple(block), kappa, phases
        self.U = U
        self.V = int(np.prod(dims))
        self.U_dev = dev(U)
        self.h = binding.mbbs_lattice_create(dims, block, self.U_dev, kappa, phases)

    def close(self):
        if self.h is not None:
            binding.mbbs_lattice_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def flush(msg):
    print(msg, flush=True)
