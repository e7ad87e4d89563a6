"""The batched evaluation that allocates nothing (reaxff_compute_forces_batched).

Called through the C ABI twice in a row, the second time on a smaller batch
(fewer clusters, a smaller largest cluster), and checked against the planned
batched evaluation (reaxff_batch_compute) of the same clusters: every energy
term of every cluster and every force to 1e-9 relative, status words clear.
A third call with a cluster longer than max_atoms checks the size report.
"""
import numpy as np
import pytest

import reaxff_synth as rs

pytestmark = pytest.mark.gpu

INT32_MAX = 2 ** 31 - 1


def _dev(pos, typ, q, off):
    import torch
    d = torch.device("cuda:0")
    return (torch.tensor(pos, dtype=torch.float64, device=d).reshape(-1, 3).contiguous(),
            torch.tensor(typ, dtype=torch.int32, device=d).contiguous(),
            torch.tensor(q, dtype=torch.float64, device=d).contiguous(),
            torch.tensor(off, dtype=torch.int64, device=d).contiguous())


def _planned(ff, P, T, Q, off):
    from paper_1706_07772_amd import Batch
    b = Batch(ff, off, (128, 2, 8))
    f, e = b.compute(P, T, Q)
    rc, bad = b.status()
    out = f.cpu().numpy(), e.cpu().numpy()
    b.close()
    assert rc == 0 and bad == -1
    return out


def _check(f, e, f_ref, e_ref, off):
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(f))
    scale = np.maximum(np.abs(e_ref).sum(axis=1, keepdims=True), 1.0)
    assert np.all(np.abs(e - e_ref) <= 1e-9 * scale), np.abs(e - e_ref).max()
    fmax = max(np.abs(f_ref).max(), 1.0)
    assert np.abs(f - f_ref).max() <= 1e-9 * fmax


def test_no_alloc_batched_matches_planned():
    import torch
    from paper_1706_07772_amd import ReaxFF
    params = rs.draw_params(0)
    ff = ReaxFF(params)
    try:
        for nsys, seed, lo, hi in ((300, 11, 10, 300), (40, 12, 1, 120)):
            pos, typ, q, off = rs.cluster_batch(nsys, seed=seed, lo=lo, hi=hi)
            max_atoms = int(np.diff(off).max())
            print(f"no-alloc batch: {nsys} clusters, {int(off[-1])} atoms, max {max_atoms}", flush=True)
            P, T, Q, O = _dev(pos, typ, q, off)
            f_ref, e_ref = _planned(ff, P, T, Q, off)
            f, e, st = ff.compute_forces_batched(O, max_atoms, P, T, Q)
            torch.cuda.synchronize()
            s = st.cpu().numpy()
            assert s[0] == 0 and s[2] == INT32_MAX, s
            _check(f.cpu().numpy(), e.cpu().numpy(), f_ref, e_ref, off)
        # a cluster longer than the stated bound is reported, the others still evaluated
        pos, typ, q, off = rs.cluster_batch(12, seed=13, lo=10, hi=60)
        sizes = np.diff(off)
        big = int(np.argmax(sizes))
        P, T, Q, O = _dev(pos, typ, q, off)
        f_ref, e_ref = _planned(ff, P, T, Q, off)
        f, e, st = ff.compute_forces_batched(O, int(sizes[big]) - 1, P, T, Q)
        torch.cuda.synchronize()
        s = st.cpu().numpy()
        e = e.cpu().numpy()
        bad = sizes > sizes[big] - 1
        assert s[0] & 4 and s[2] == int(np.flatnonzero(bad)[0]), s
        assert np.all(np.isnan(e[bad]))
        ok = ~bad
        scale = np.maximum(np.abs(e_ref[ok]).sum(axis=1, keepdims=True), 1.0)
        assert np.all(np.abs(e[ok] - e_ref[ok]) <= 1e-9 * scale)
    finally:
        ff.close()


def test_no_alloc_batched_rejects_bad_arguments():
    import torch
    from paper_1706_07772_amd import ReaxFF, ReaxFFError
    ff = ReaxFF(rs.draw_params(0))
    try:
        pos, typ, q, off = rs.cluster_batch(4, seed=14, lo=10, hi=40)
        P, T, Q, O = _dev(pos, typ, q, off)
        for bad_max in (0, 385):
            with pytest.raises(ReaxFFError) as ei:
                ff.compute_forces_batched(O, bad_max, P, T, Q)
            assert ei.value.code == -1
        # no clusters: nothing to do, status cleared
        O0 = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        _, e, st = ff.compute_forces_batched(O0, 1, P, T, Q)
        torch.cuda.synchronize()
        assert e.shape == (0, 12) and st.cpu().numpy()[0] == 0
    finally:
        ff.close()
