"""hgp_eri_prim_quartets_noalloc (the entry point for callers that cannot
allocate device memory) against hgp_eri_prim_quartets, through the C ABI:
two calls in a row per class, the second with fewer quartets, each compared
element by element with the allocating entry point's result."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

# register-tier and staged-tier classes (the tiers the fixed buffer serves)
CASES = [((0, 0, 0, 0), 6000, 1500), ((2, 1, 1, 0), 5000, 1200), ((1, 2, 0, 1), 3000, 800),
         ((2, 2, 2, 2), 3000, 700), ((2, 1, 2, 2), 2500, 300)]


@pytest.mark.parametrize("ls,n1,n2", CASES)
def test_noalloc_matches_allocating_entry(ls, n1, n2):
    import torch
    import paper_2605_10312_amd as hgp
    torch.cuda.set_device(0)
    assert hgp.eri_prim_quartets_noalloc_max(ls) >= n1
    nsph = int(np.prod([2 * l + 1 for l in ls]))
    for call, n in enumerate((n1, n2)):
        cen, ex = workloads.prim_quartets(max(ls), n, seed=7000 + call)
        ct = torch.tensor(cen, device="cuda")
        et = torch.tensor(ex, device="cuda")
        ref = torch.empty((n, nsph), dtype=torch.float64, device="cuda")
        got = torch.full((n, nsph), float("nan"), dtype=torch.float64, device="cuda")
        print(f"noalloc: class {ls}, call {call}, n {n}", flush=True)
        hgp.eri_prim_quartets(ls, ct, et, ref)
        hgp.eri_prim_quartets_noalloc(ls, ct, et, got)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(g).all()
        err = float(np.abs(g - r).max())
        print(f"  max |noalloc - alloc| = {err:.3e} (identical: {np.array_equal(g, r)})", flush=True)
        assert err <= 1e-12


def test_noalloc_rejects_beyond_its_buffer():
    import torch
    import paper_2605_10312_amd as hgp
    ls = (2, 2, 2, 2)
    nmax = hgp.eri_prim_quartets_noalloc_max(ls)
    assert nmax > 0
    ct = torch.zeros((nmax + 1, 4, 3), dtype=torch.float64, device="cuda")
    et = torch.ones((nmax + 1, 4), dtype=torch.float64, device="cuda")
    out = torch.empty((nmax + 1, 625), dtype=torch.float64, device="cuda")
    with pytest.raises(hgp.HGPError) as ei:
        hgp.eri_prim_quartets_noalloc(ls, ct, et, out)
    assert ei.value.status == -1
