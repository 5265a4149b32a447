"""GPU multi-RHS Wilson-Dirac operator against the oracle (Sec. 2.1).

Small lattices: every element, several L (including ones that do not fill a
column chunk), twisted boundary phases.  Full 32^3 x 64, L = 12 (the
benchmark's workload and launch configuration): sampled sites, boundary
sites included, checked one by one with the oracle's per-site form.
Tolerances (per column, norm-wise relative): FP64 1e-14, FP32 1e-6,
FP16 storage 2e-3.
"""

import numpy as np
import pytest

from oracle import dirac, geometry
from paper_1104_0737_amd import configs, inputs

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
torch = gu.torch
B = gu.binding

PH_TWIST = ((np.cos(0.3), np.sin(0.3)), (1.0, 0.0), (np.cos(1.1), -np.sin(1.1)), (-1.0, 0.0))
TOL = {B.FP64: 1e-14, B.FP32: 1e-6, B.FP16S: 2e-3}


@pytest.mark.parametrize("dims,block,L", [((4, 4, 4, 4), (2, 2, 2, 2), 1), ((4, 4, 4, 6), (2, 2, 2, 3), 5),
                                          ((8, 8, 8, 8), (4, 4, 4, 4), 4), ((4, 6, 4, 8), (2, 3, 2, 4), 12),
                                          ((8, 4, 4, 4), (4, 2, 2, 2), 7)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_dslash_parity(dims, block, L, prec):
    gu.flush(f"dslash {dims} L={L} prec={prec}")
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.35, 11)
    X = inputs.gaussian_block(V, L, 12)
    ref = dirac.apply_D(U, 0.1235, PH_TWIST, X, dims).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.1235, PH_TWIST) as lat:
        Xd = gu.dev(X)
        Yd = torch.empty_like(Xd)
        B.mbbs_apply_dirac(lat.h, L, Xd, Yd, prec)
        Y = gu.host(Yd)
        err = gu.rel_col_err(Y, ref)
        emax = gu.max_elem_err(Y, ref)
    assert np.all(err <= TOL[prec]), err
    assert np.all(emax <= TOL[prec]), emax


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_blocked_operator_parity(prec):
    dims, block, L = (8, 8, 4, 4), (4, 4, 2, 2), 3
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.3, 13)
    X = inputs.gaussian_block(V, L, 14)
    ref = dirac.apply_blocked(U, 0.12, PH_TWIST, X, dims, block).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.12, PH_TWIST) as lat:
        Xd = gu.dev(X)
        Yd = torch.empty_like(Xd)
        B.mbbs_apply_blocked(lat.h, L, Xd, Yd, prec)
        Y = gu.host(Yd)
        err = gu.rel_col_err(Y, ref)
        emax = gu.max_elem_err(Y, ref)
    assert np.all(err <= TOL[prec]), err
    assert np.all(emax <= TOL[prec]), emax


def test_point_source_and_zero_columns():
    # a point source exercises FP16 per-site scales (most sites are zero)
    dims, block, L = (4, 4, 4, 4), (2, 2, 2, 2), 4
    V = 256
    U = inputs.gauge_field(dims, 0.3, 15)
    X = inputs.point_sources(V, L, 37, 2)
    X[:, 3] = 0
    ref = dirac.apply_D(U, 0.13, gu.PH_AP, X, dims).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.13) as lat:
        for prec in (0, 1, 2):
            Yd = torch.empty((12 * V, L), dtype=torch.complex128, device="cuda")
            B.mbbs_apply_dirac(lat.h, L, gu.dev(X), Yd, prec)
            Y = gu.host(Yd)
            assert np.all(Y[:, 3] == 0)
            err = gu.rel_col_err(Y[:, :3], ref[:, :3])
            assert np.all(err <= TOL[prec]), (prec, err)


def test_deterministic_repeat():
    dims, L = (8, 8, 8, 8), 12
    V = 4096
    U = inputs.gauge_field(dims, 0.3, 16)
    with gu.Lattice(dims, (4, 4, 4, 4), U, 0.11) as lat:
        Xd = gu.dev(inputs.gaussian_block(V, L, 17))
        outs = []
        for _ in range(3):
            Yd = torch.empty_like(Xd)
            B.mbbs_apply_dirac(lat.h, L, Xd, Yd, 0)
            outs.append(gu.host(Yd))
    assert outs[0].tobytes() == outs[1].tobytes() == outs[2].tobytes()


def _sample_sites(dims, n, seed):
    rng = np.random.default_rng(seed)
    c = [[0, 0, 0, 0], [d - 1 for d in dims], [dims[0] - 1, 0, dims[2] - 1, 0], [0, dims[1] - 1, 0, dims[3] - 1]]
    sites = [int(geometry.site_of(dims, x)) for x in c]
    sites += rng.integers(0, int(np.prod(dims)), n).tolist()
    return np.array(sites)


@pytest.mark.slow
def test_dslash_full_size_sampled():
    """32^3 x 64, L = 12, FP64, FP32 and FP16 storage, in the default launch
    settings and in those the benchmark's tuning chose (its recorded JSON
    line), at sampled sites; FP64 also on two whole columns."""
    cfg = configs.c4()
    dims, L = cfg.dims, 12
    V = cfg.V
    gu.flush("full-size: generating links")
    U = cfg.gauge()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4004)
    with gu.Lattice(dims, cfg.block, U, cfg.kappa) as lat:
        Xd = torch.randn((12 * V, L), dtype=torch.complex128, device="cuda", generator=gen)
        sites = _sample_sites(dims, 200, 4005)
        X = gu.host(Xd)
        ref = dirac.apply_D_sites(U, cfg.kappa, cfg.phases, X.reshape(V, 4, 3, L), dims, sites)
        idx = torch.from_numpy((12 * sites[:, None] + np.arange(12)[None, :]).ravel()).cuda()
        Yd = torch.empty_like(Xd)
        for tuned in (False, True):
            tag = "tuned settings" if tuned else "default settings"
            if tuned:
                gu.apply_benchmark_tuning(lat.h)
            gu.flush(f"full-size: FP64, {tag}")
            B.mbbs_apply_dirac(lat.h, L, Xd, Yd, B.FP64)
            got = gu.host(Yd.index_select(0, idx))
            err = gu.rel_col_err(got, ref.reshape(-1, L))
            assert np.all(err <= 1e-14), (tag, err)
            if not tuned:
                # two columns over the whole lattice, every element
                gu.flush("full-size: FP64, columns 0 and 7 over the whole lattice")
                cols = [0, 7]
                Xc = np.ascontiguousarray(X[:, cols])
                refc = dirac.apply_D(U, cfg.kappa, cfg.phases, Xc, dims).reshape(12 * V, 2)
                Yc = gu.host(Yd)[:, cols]
                assert np.all(gu.rel_col_err(Yc, refc) <= 1e-14)
                assert np.all(gu.max_elem_err(Yc, refc) <= 1e-14)
                del refc, Yc, Xc
            gu.flush(f"full-size: FP32 storage, {tag}")
            X32 = torch.empty((12 * V, L, 2), dtype=torch.float32, device="cuda")
            Y32 = torch.empty_like(X32)
            B.mbbs_convert_to(B.FP32, V, L, Xd, X32)
            B.mbbs_apply_dirac_raw(lat.h, L, B.FP32, X32, None, Y32, None)
            B.mbbs_convert_from(B.FP32, V, L, Y32, None, Yd)
            got = gu.host(Yd.index_select(0, idx))
            err = gu.rel_col_err(got, ref.reshape(-1, L))
            assert np.all(err <= 1e-6), (tag, err)
            del X32, Y32
            gu.flush(f"full-size: FP16 storage, {tag}")
            X16 = torch.empty((12 * V, L, 2), dtype=torch.float16, device="cuda")
            Y16 = torch.empty_like(X16)
            X16s = torch.empty((V, L), dtype=torch.float32, device="cuda")
            Y16s = torch.empty_like(X16s)
            B.mbbs_convert_to(B.FP16S, V, L, Xd, X16, X16s)
            B.mbbs_apply_dirac_raw(lat.h, L, B.FP16S, X16, X16s, Y16, Y16s)
            B.mbbs_convert_from(B.FP16S, V, L, Y16, Y16s, Yd)
            got = gu.host(Yd.index_select(0, idx))
            err = gu.rel_col_err(got, ref.reshape(-1, L))
            assert np.all(err <= 2e-3), (tag, err)
            assert np.all(gu.max_elem_err(got, ref.reshape(-1, L)) <= 2e-3), tag
            del X16, Y16, X16s, Y16s


def test_tuning_is_bit_identical():
    """Launch shapes, paired hops and nontemporal stores chosen by the
    autotuner never change results."""
    from paper_1104_0737_amd import autotune
    dims, L = (8, 8, 8, 8), 12
    V = 4096
    U = inputs.gauge_field(dims, 0.3, 18)
    X = gu.dev(inputs.gaussian_block(V, L, 19))
    with gu.Lattice(dims, (4, 4, 4, 4), U, 0.11) as lat:
        for prec in (0, 1, 2):
            ref = None
            settings = [c + (0, 0) for c in autotune.candidates(L, prec)] + autotune.operator_candidates(L, prec)
            # other columns per thread: another summation order
            settings = [x for x in settings if len(x) < 6 or x[5] == 0]
            for setting in settings:
                if setting[2]:
                    continue          # the split kernels sum the hops in another order
                autotune.apply(lat.h, prec, setting)
                Y = torch.empty_like(X)
                B.mbbs_apply_dirac(lat.h, L, X, Y, prec)
                out = gu.host(Y)
                if ref is None:
                    ref = out
                assert out.tobytes() == ref.tobytes(), (prec, setting)


@pytest.mark.parametrize("split", [2, 4])
@pytest.mark.parametrize("L", [4, 12, 5])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_split_wave_parity(split, L, prec):
    """Hops split over wave groups (L = 5 has no split shape: falls back)."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    V = 4096
    U = inputs.gauge_field(dims, 0.35, 20)
    X = inputs.gaussian_block(V, L, 21)
    ref = dirac.apply_D(U, 0.1235, PH_TWIST, X, dims).reshape(12 * V, L)
    refb = dirac.apply_blocked(U, 0.1235, PH_TWIST, X, dims, block).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.1235, PH_TWIST) as lat:
        B.mbbs_lattice_tune(lat.h, B.TUNE_SPLIT[prec], split)
        Xd = gu.dev(X)
        Yd = torch.empty_like(Xd)
        B.mbbs_apply_dirac(lat.h, L, Xd, Yd, prec)
        assert np.all(gu.rel_col_err(gu.host(Yd), ref) <= TOL[prec])
        B.mbbs_apply_blocked(lat.h, L, Xd, Yd, prec)
        assert np.all(gu.rel_col_err(gu.host(Yd), refb) <= TOL[prec])


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_operator_wide_block(prec):
    """L = 64 (the operator's largest block) and L = 16 with every columns-per-thread setting."""
    dims, block = (4, 4, 4, 8), (2, 2, 2, 4)
    V = 512
    U = inputs.gauge_field(dims, 0.35, 22)
    for L, chunks in ((64, (0,)), (16, (1, 2, 4))):
        X = inputs.gaussian_block(V, L, 23)
        ref = dirac.apply_D(U, 0.12, PH_TWIST, X, dims).reshape(12 * V, L)
        with gu.Lattice(dims, block, U, 0.12, PH_TWIST) as lat:
            for ch in chunks:
                B.mbbs_lattice_tune(lat.h, B.TUNE_CHUNK[prec], ch)
                Xd = gu.dev(X)
                Yd = torch.empty_like(Xd)
                B.mbbs_apply_dirac(lat.h, L, Xd, Yd, prec)
                assert np.all(gu.rel_col_err(gu.host(Yd), ref) <= TOL[prec]), (L, ch)


def test_block_threads_per_precision():
    """Threads per block can be set for one precision's kernels alone (out of
    range values are rejected); every value leaves the result bits unchanged,
    and the all-precision knob still applies to every precision."""
    dims, L = (8, 8, 8, 8), 12
    V = 4096
    U = inputs.gauge_field(dims, 0.3, 24)
    X = gu.dev(inputs.gaussian_block(V, L, 25))
    with gu.Lattice(dims, (4, 4, 4, 4), U, 0.11) as lat:
        for bad in (31, 257):
            with pytest.raises(B.MbbsError) as e:
                B.mbbs_lattice_tune(lat.h, B.TUNE_BLOCK_THREADS_PREC[1], bad)
            assert e.value.code == B.EINVAL
        with pytest.raises(B.MbbsError):
            B.mbbs_lattice_tune(lat.h, 99, 128)            # no such knob
        for prec in (0, 1, 2):
            Y = torch.empty_like(X)
            B.mbbs_apply_dirac(lat.h, L, X, Y, prec)
            ref = gu.host(Y)
            for t in (64, 96, 192):
                B.mbbs_lattice_tune(lat.h, B.TUNE_BLOCK_THREADS_PREC[prec], t)
                B.mbbs_lattice_tune(lat.h, B.TUNE_BLOCK_THREADS_PREC[(prec + 1) % 3], 256 - t)
                B.mbbs_apply_dirac(lat.h, L, X, Y, prec)
                assert gu.host(Y).tobytes() == ref.tobytes(), (prec, t)
            B.mbbs_lattice_tune(lat.h, B.TUNE_BLOCK_THREADS, 128)
            B.mbbs_apply_dirac(lat.h, L, X, Y, prec)
            assert gu.host(Y).tobytes() == ref.tobytes(), prec
