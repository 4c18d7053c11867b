"""vfp_reconstruct (f at every basis node in given directions) against the
oracle's sum over the coefficients; ragged row and direction tiles."""

import math

import numpy as np
import pytest

from oracle import sh
from paper_2501_05110_amd import workloads as W

from gpu_cases import _say, rel_inf, shock

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wl_args,ndir,offset", [((13, 9, 2, 1), 50, 0), ((9, 5, 2, 7), 33, 0),
                                                 ((11, 6, 1, 5), 1, 0), ((14, 7, 2, 3), 64, 0),
                                                 ((14, 7, 2, 3), 64, 1), ((10, 3, 1, 3), 130, 0),
                                                 ((14, 7, 2, 3), 16, 0), ((13, 9, 2, 1), 7, 1),
                                                 ((11, 6, 1, 5), 16, 1), ((9, 5, 2, 7), 12, 0)])
def test_reconstruct_parity(lib, cuda, wl_args, ndir, offset):
    """Even ndir writes direction pairs with 16-byte stores; odd ndir, or an
    output that starts 8 bytes past a 16-byte boundary (offset 1), takes the
    8-byte stores; 130 directions span three direction tiles; up to 16
    directions (n <= 49) take the 16-direction workgroups with 128-row
    tiles, and l_max = 7 with 12 directions the 64-direction ones."""
    import torch
    from paper_2501_05110_amd import vfp
    wl = shock(*wl_args)
    op = vfp.Operator(wl)
    rng = np.random.default_rng(12)
    th, ph = np.arccos(rng.uniform(-1, 1, ndir)), rng.uniform(0, 2 * math.pi, ndir)
    z = W.random_state(wl, 3)
    Y = torch.from_numpy(vfp.sh_eval(wl.lmax, th, ph)).cuda()
    rows = wl.ndofs // wl.n_lms
    buf = torch.full((rows * ndir + 2,), 7.0, dtype=torch.float64, device="cuda")
    out = buf[offset:offset + rows * ndir]
    op.reconstruct(torch.from_numpy(z.ravel()).cuda(), Y, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(rows, ndir)
    rest = np.delete(buf.cpu().numpy(), np.arange(offset, offset + rows * ndir))
    assert np.all(rest == 7.0)          # nothing written outside out
    want = sh.reconstruct(z, wl.lmax, th, ph)
    err = rel_inf(got, want)
    _say(f"[reconstruct] {wl.name} rows={rows} ndir={ndir} offset={offset} rel_inf={err:.2e}")
    assert err <= 1e-13
