"""Helpers shared by the GPU tests: device tensors and lattice handles."""

import os

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


def apply_benchmark_tuning(h):
    """The launch settings the benchmark's tuning chose at this size (its
    recorded JSON line): each precision's operator setting, then its SAP
    setting (tiled MR stencil and residual, psi formed once, ...)."""
    import json
    from paper_1104_0737_amd import autotune
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "tuning_32x32x32x64_L12.txt")
    with open(path) as f:
        tun = json.loads(f.read().strip().splitlines()[-1])["tuning"]
    for prec, name in ((binding.FP64, "fp64"), (binding.FP32, "fp32"), (binding.FP16S, "fp16s")):
        t = tun[name]
        autotune.apply(h, prec, (t["group_cols"], t["block_threads"], t["split"], t["hop_pair"], t["nt_store"],
                                 t.get("chunk", 0), t.get("tile", 0), 0, t.get("tile_cols", 0)))
        if "sap" in t:
            autotune.apply(h, prec, tuple(t["sap"]["setting"]))
    flush(f"  tuned settings: fp32 SAP {tun['fp32']['sap']['setting']}, fp16s SAP {tun['fp16s']['sap']['setting']}")
