"""A lattice whose 27 population planes pass 2^32 elements (576x576x512,
170M cells, 18 GB per population buffer): the plane offsets of the pull, the
stores and the canonical read-back must not wrap. One step from a smooth
non-uniform equilibrium (f_i(y, 0) = f^eq_i(rho0(y), u0(y))), checked on
sampled cells -- among them the last cells, whose upper planes lie past 2^32
elements: f_i(x, 1) is the oracle's collision at y = x - c_i, component i
(the oracle cannot hold the whole lattice in a test)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import say

pytestmark = pytest.mark.gpu

NX, NY, NZ = 576, 576, 512
TAU = 0.7


def _fields(dev):
    """rho0 (nz, ny, nx) and u0 (3, nz, ny, nx), smooth, made on the device."""
    z = torch.arange(NZ, device=dev, dtype=torch.float32).view(NZ, 1, 1) * (2 * np.pi / NZ)
    y = torch.arange(NY, device=dev, dtype=torch.float32).view(1, NY, 1) * (2 * np.pi / NY)
    x = torch.arange(NX, device=dev, dtype=torch.float32).view(1, 1, NX) * (2 * np.pi / NX)
    rho = 1.0 + 0.01 * torch.sin(x + 0.3) * torch.cos(2 * y) * torch.sin(z - 0.7)
    full = (NZ, NY, NX)
    u = torch.stack([(0.03 * torch.sin(y + z)).expand(full), (-0.02 * torch.cos(x - 2 * z)).expand(full),
                     (0.025 * torch.sin(3 * x + y)).expand(full)])
    return rho.contiguous(), u.contiguous()


def test_one_step_past_2_to_the_32_population_elements():
    from paper_2206_01683_amd import lbm
    dev = torch.device("cuda")
    ncell = NX * NY * NZ
    assert 27 * ncell > 2 ** 32
    rho0, u0 = _fields(dev)
    sim = lbm.Simulation(NX, NY, NZ, TAU, rho0=rho0, u0=u0)
    sim.step(np.zeros((1, 18)))
    assert sim.check() == 0
    f1 = sim.read_populations()  # canonical pre-collision f_i(x, 1) = f*_i(x - c_i, 0)
    C, _ = oracle.lattice()
    rng = np.random.default_rng(7)
    cells = np.concatenate([[ncell - 1, ncell - 2, ncell - NX, ncell - NX * NY, 0, 1],
                            rng.integers(0, ncell, 60)])
    zc, yc, xc = np.unravel_index(cells, (NZ, NY, NX))
    # the cells whose collision feeds a sampled cell: y = x - c_i; the initial
    # pre-collision populations there are f^eq(rho0(y), u0(y))
    zu = torch.as_tensor(np.stack([(zc - C[i, 2]) % NZ for i in range(27)]), device=dev)
    yu = torch.as_tensor(np.stack([(yc - C[i, 1]) % NY for i in range(27)]), device=dev)
    xu = torch.as_tensor(np.stack([(xc - C[i, 0]) % NX for i in range(27)]), device=dev)
    r_up = rho0[zu, yu, xu].double().cpu().numpy()
    u_up = torch.stack([u0[a][zu, yu, xu] for a in range(3)]).double().cpu().numpy()
    frame = np.zeros(18)
    want = np.zeros((27, len(cells)))
    for k in range(len(cells)):
        for i in range(27):
            fin = oracle.equilibrium(r_up[i, k], u_up[:, i, k])
            out, _, _ = oracle.collide_node(fin, np.zeros(3), frame, np.zeros(3), TAU)
            want[i, k] = out[i]
    got = torch.stack([f1[i][torch.as_tensor(zc, device=dev), torch.as_tensor(yc, device=dev),
                              torch.as_tensor(xc, device=dev)] for i in range(27)]).double().cpu().numpy()
    err = np.abs(got - want).max()
    say(f"{NX}x{NY}x{NZ} ({27 * ncell / 2 ** 32:.2f} x 2^32 population elements): max |df| on "
        f"{len(cells)} sampled cells = {err:.3e}")
    assert err < 1e-6 * np.abs(want).max()
    del f1
    sim.close()
    torch.cuda.empty_cache()
