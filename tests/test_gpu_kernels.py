"""GPU parity of single steps of the path against the oracle: Fermi-Dirac
integrals, the 3D real/complex FFT, structure factor and ionic field."""
import math
import sys

import numpy as np
import pytest

from oracle import fd as ofd
from oracle import ionic as oion
from oracle import scf as oscf
from oracle.grid import Grid
from paper_2606_13283_amd import arche
from paper_2606_13283_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    arche.load()
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_fermi_dirac_kernel(torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(-100, 1000, 20000), rng.uniform(-3, 62, 20000),
                        np.array([-2.0, -2.0 + 1e-15, 60.0, 60.0 - 1e-13, 0.0, -745.0])])
    say("fd kernel n=%d" % x.size)
    a, b, c = arche.fermi_dirac(torch.from_numpy(x).cuda())
    ref = ofd.fd_integrals(x)
    for got, name in ((a, "m12"), (b, "p12"), (c, "p32")):
        g = got.cpu().numpy()
        r = ref[name]
        m = r > 1e-300
        rel = np.abs(g[m] - r[m]) / r[m]
        assert rel.max() <= 5e-15, (name, x[m][np.argmax(rel)], rel.max())


def test_fermi_dirac_derivatives(torch_cuda):
    """The SCF kernel's I_{1/2} and derivatives: the first is I_{-1/2}/2 exactly
    (dI_j/dx = j I_{j-1}); the second and third against central differences of
    the oracle's I_{-1/2}/2 (step 1e-3: truncation about 1e-7 and 1e-5 relative);
    across all three regimes and their seams."""
    torch = torch_cuda
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(-30, 100, 6000), rng.uniform(-3, 62, 6000),
                        np.array([-2.0, -2.0 + 1e-12, -2.0 - 1e-12, 60.0, 60.0 - 1e-12, 0.0, -1.5])])
    say("fd derivs n=%d" % x.size)
    d = [t.cpu().numpy() for t in arche.fermi_dirac_derivs(torch.from_numpy(x).cuda())]
    ref = ofd.fd_integrals(x)
    h = 1e-3
    rp, rm = ofd.fd_integrals(x + h), ofd.fd_integrals(x - h)
    half = 0.5 * ref["m12"]
    assert np.max(np.abs(d[0] / ref["p12"] - 1)) <= 5e-15
    assert np.max(np.abs(d[1] / half - 1)) <= 5e-15
    r2 = 0.5 * (rp["m12"] - rm["m12"]) / (2 * h)
    r3 = 0.5 * (rp["m12"] - 2 * ref["m12"] + rm["m12"]) / h ** 2
    e2 = np.abs(d[2] - r2) / (np.abs(r2) + 1e-6 * half)
    e3 = np.abs(d[3] - r3) / (np.abs(r3) + 1e-6 * half)
    say("d2 %.2e d3 %.2e" % (e2.max(), e3.max()))
    assert e2.max() <= 1e-6 and e3.max() <= 1e-4


FFT_SHAPES = [(16, 16, 16), (32, 32, 32), (20, 24, 30), (48, 50, 54), (60, 64, 72), (128, 128, 128), (12, 18, 10),
              (192, 96, 40)]


@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_fft_roundtrip_vs_numpy(torch_cuda, shape):
    torch = torch_cuda
    say("fft shape", shape)
    rng = np.random.default_rng(sum(shape))
    f = rng.standard_normal(shape)
    X = arche.fft_r2c(torch.from_numpy(f).cuda()).cpu().numpy()
    ref = np.fft.rfftn(f)
    assert np.max(np.abs(X - ref)) <= 5e-14 * np.max(np.abs(ref)) * math.log2(np.prod(shape))
    # inverse of an arbitrary (non-Hermitian on the self-conjugate planes) half spectrum
    H = rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)
    y = arche.fft_c2r(torch.from_numpy(H).cuda(), shape[2]).cpu().numpy()
    yref = np.fft.irfftn(H, s=shape, axes=(0, 1, 2)) * np.prod(shape)
    assert np.max(np.abs(y - yref)) <= 5e-14 * np.max(np.abs(yref)) * math.log2(np.prod(shape))


@pytest.mark.parametrize("var", [1, 2, 0])
def test_fft_tile_variants(torch_cuda, var):
    """Every tile variant of the tunable line lengths is the same transform."""
    torch = torch_cuda
    L = arche.load()
    shape = (100, 120, 128)
    for pas, n in ((0, shape[1]), (1, shape[0]), (2, shape[2])):
        assert L.arche_fft_tile(pas, n, var) == var
    say("fft tile variant", var, shape)
    rng = np.random.default_rng(var)
    f = rng.standard_normal(shape)
    X = arche.fft_r2c(torch.from_numpy(f).cuda()).cpu().numpy()
    ref = np.fft.rfftn(f)
    assert np.max(np.abs(X - ref)) <= 5e-14 * np.max(np.abs(ref)) * math.log2(np.prod(shape))
    H = rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)
    y = arche.fft_c2r(torch.from_numpy(H).cuda(), shape[2]).cpu().numpy()
    yref = np.fft.irfftn(H, s=shape, axes=(0, 1, 2)) * np.prod(shape)
    assert np.max(np.abs(y - yref)) <= 5e-14 * np.max(np.abs(yref)) * math.log2(np.prod(shape))


def _ctx_and_oracle(w, opts=None):
    ctx = arche.Context.from_workload(w, opts)
    s = oscf.System(w.cell, w.grid, w.pos, w.species, w.Z, w.rc, w.mass, w.kT, w.lam, w.xc)
    return ctx, s


def _mirror(a):
    """a[-m mod N] on the full box"""
    return np.roll(np.flip(a, axis=(0, 1, 2)), 1, axis=(0, 1, 2))


@pytest.mark.parametrize("case", ["fcc32", "ortho2sp"])
def test_structure_factor_and_ionic_field(torch_cuda, case):
    if case == "fcc32":
        w = W.fcc32()
    else:
        w = W.small_random(10, 16, 2.7, 5.0, seed=3, shape=(16, 20, 24), stretch=(1.0, 1.2, 1.4))
        w.species = np.array([0, 1] * 5, dtype=np.int32)
        w.Z, w.rc, w.mass = (3.0, 1.0), (1.1, 0.6), (W.AL_MASS, 1837.0)
    say("structure factor", w.name)
    ctx, s = _ctx_and_oracle(w, arche.Options(scf_max_iter=1))
    ctx.solve(w.pos, allow_noconv=True)
    ion = oscf.ionic_setup(s)
    Nz = w.grid[2]
    Sp = ctx.debug("SZ_plus")
    Sm = ctx.debug("SZ_minus")
    ref = ion.SZ[:, :, : Nz // 2 + 1]
    scale = np.max(np.abs(ion.SZ))
    assert np.max(np.abs(Sp - ref)) <= 1e-12 * scale
    refm = np.conj(_mirror(ion.SZ))[:, :, : Nz // 2 + 1]
    assert np.max(np.abs(Sm - refm)) <= 1e-12 * scale
    Vie = ctx.debug("Vie")
    assert np.max(np.abs(Vie - ion.Vie)) <= 1e-12 * np.max(np.abs(ion.Vie))
    ctx.close()
