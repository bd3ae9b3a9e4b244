"""The allocation-free SITE entry point (siting_greedy_noalloc), called
through the C ABI with caller-owned outputs, against siting_greedy on the same
inputs: two calls in a row on one device, the second with fewer candidates and
a smaller terrain (so a stale state from the first call would show), each
checked output for output (selection, gains, count, cumulative viewshed)
against the workspace entry point and against the oracle's greedy."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[no-alloc]", *a, flush=True)


def _case(orc, seed, nr, nc, n_obs, roi, max_obs, frac):
    from synth import fbm, uniform_observers
    z = fbm(nr, 2.4, 1500, seed, ncols=nc)
    obs = uniform_observers(nr, nc, n_obs, seed, roi=roi, height=(5, 40))
    bm, off = orc.viewshed(z, obs)
    tgt = nr * nc if frac >= 1 else int(math.ceil(frac * nr * nc))
    return obs, bm, off, tgt


def test_greedy_noalloc_matches_workspace_entry_point(orc):
    import paper_2006_16783_amd as S
    from paper_2006_16783_amd import _lib as L
    assert torch.cuda.is_available()
    cases = [(21, 700, 650, 2500, (10, 160), 300, 1.0),   # windows above 1024 words too
             (22, 300, 280, 400, (5, 60), 120, 0.6)]      # then a smaller input
    for seed, nr, nc, n_obs, roi, max_obs, frac in cases:
        _say("case", seed, nr, nc, n_obs, roi, max_obs, frac)
        obs, bm_h, off, tgt = _case(orc, seed, nr, nc, n_obs, roi, max_obs, frac)
        wsel, wgain, wcum, _ = orc.greedy(bm_h, off, obs, nr, nc, max_obs, tgt, lazy=True)
        bm = torch.from_numpy(bm_h.view(np.int64)).cuda()
        off_d = torch.from_numpy(off).cuda()
        obs_d = S.observers_to_device(obs)
        # the workspace entry point
        sel, gains, nsel, cum = S.siting_greedy(bm, off_d, obs_d, nr, nc, max_obs, tgt)
        # the allocation-free one, outputs preset to garbage so that every
        # value it reports is its own
        W = (nc + 63) // 64
        cum2 = torch.full((nr, W), -1, dtype=torch.int64, device="cuda")
        sel2 = torch.full((max_obs,), -7, dtype=torch.int64, device="cuda")
        gains2 = torch.full((max_obs,), -7, dtype=torch.int64, device="cuda")
        nsel2 = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        rc = L.lib().siting_greedy_noalloc(
            bm.data_ptr(), off_d.data_ptr(), obs_d.data_ptr(), len(obs), nr, nc, max_obs, tgt,
            cum2.data_ptr(), sel2.data_ptr(), gains2.data_ptr(), nsel2.data_ptr(), stream)
        assert rc == 0, L.last_error()
        torch.cuda.synchronize()
        m, m2 = int(nsel.item()), int(nsel2.item())
        assert m == m2 == len(wsel)
        assert (sel2[:m].cpu().numpy() == sel[:m].cpu().numpy()).all()
        assert (gains2[:m].cpu().numpy() == gains[:m].cpu().numpy()).all()
        assert (sel2[:m].cpu().numpy() == wsel).all() and (gains2[:m].cpu().numpy() == wgain).all()
        # entries past nselected are left untouched
        assert (sel2[m:].cpu().numpy() == -7).all()
        assert torch.equal(cum2, cum)
        assert (cum2.cpu().numpy().view(np.uint64).reshape(-1) == wcum.reshape(-1)).all()
        _say("equal:", m, "selections")
