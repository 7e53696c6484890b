"""sh_projectors_noalloc (the projector build for callers that cannot allocate)
against sh_radial_create + sh_projectors / sh_projectors_f32 on the same inputs,
bit for bit.  Two calls in a row per dtype, the second smaller than the first (the
static working buffer keeps the first call's contents), then a call whose tables
exceed the buffer, which must be refused before anything is launched."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2510_05282_amd as sh
from paper_2510_05282_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(seed, n_atoms, lmax, h):
    A = workloads.atom_spheres(seed=seed, n_atoms=n_atoms, radius=2.0, h=h, lmax=lmax, n_r=2000)
    return A


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_noalloc_matches_handle_path(dev, dt):
    ref_fn = sh.sh_projectors if dt == torch.float64 else sh.sh_projectors_f32
    for seed, n_atoms, lmax, h in ((1, 24, 6, 0.2), (2, 5, 2, 0.3)):  # the second call is smaller
        A = _case(seed, n_atoms, lmax, h)
        print(f"case: noalloc, {n_atoms} atoms, lmax {lmax}, {int(A.offsets[-1])} points, {dt}", flush=True)
        c = torch.from_numpy(A.centers).to(dev, dt)
        off = torch.from_numpy(A.offsets).to(dev)
        p = torch.from_numpy(A.points).to(dev, dt)
        vals = torch.from_numpy(np.ascontiguousarray(A.tables)).to(dev)
        toa = torch.from_numpy(np.arange(n_atoms)[::-1].copy().astype(np.int32)).to(dev)
        F = (lmax + 1) ** 2
        out = torch.full((F * p.shape[0],), float("nan"), dtype=dt, device=dev)
        got = sh.sh_projectors_noalloc(lmax, c, off, p, vals, A.r_max, table_of_atom=toa, out=out)
        rad = sh.Radial(A.tables, A.r_max)
        ref = ref_fn(lmax, c, off, p, rad, table_of_atom=toa)
        rad.close()
        assert torch.equal(got, ref)


def test_noalloc_refuses_oversized_tables(dev):
    lmax, n_r = 9, 2000
    n_tables = (2 ** 21) // ((lmax + 1) * n_r) + 1  # one table more than the buffer holds
    vals = torch.zeros((n_tables, lmax + 1, n_r), dtype=torch.float64, device=dev)
    c = torch.zeros((1, 3), dtype=torch.float64, device=dev)
    off = torch.tensor([0, 4], dtype=torch.int64, device=dev)
    p = torch.ones((4, 3), dtype=torch.float64, device=dev)
    out = torch.zeros(100 * 4, dtype=torch.float64, device=dev)
    with pytest.raises(sh.ShError) as e:
        sh.sh_projectors_noalloc(lmax, c, off, p, vals, 3.0, out=out)
    assert e.value.code == 1  # SH_EINVAL
    assert torch.count_nonzero(out) == 0
