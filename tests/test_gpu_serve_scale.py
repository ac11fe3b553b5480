"""Serving at full size: the 2^30-base index (uniform ACGT with 1000 planted 10-kb segments x20 at 1 %
substitutions), built on the device with the 12-character start table, served by the native loop in
the launch configuration the benchmark times (4 slots, 256 MiB arena, batches of up to 2^18
patterns, live free-memory check) at 10^7 patterns/s. The suffix array behind the index is handed
out by the device input preparation and checked by the oracle directly; every served count then
equals the oracle's suffix-array binary search over the text, one direct count of all patterns, and
each sampled request counted alone, and so does the direct count of every pattern by the same index
over each other QuadRank layout (16-bit paired, 32-bit, 64-bit, 24/8); sampled patterns are also
recounted by the oracle's direct scan of the text."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def test_native_serve_2e30_sampled():
    qr = require_gpu()
    from paper_2602_04103_amd.serve import NativeServer, make_workload
    n = 1 << 30
    text = datagen.dna_codes(3030, n)
    datagen.plant_repeats(3031, text, nseg=1000, seglen=10_000, copies=20, sub=0.01)
    announce("serve-2^30 index")
    d_sa = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    bwt, dollar, _, _ = qr.quadfm_index_device(torch.from_numpy(text).cuda(), 0, sa=d_sa)
    fm = qr.QuadFm(bwt, n + 1, dollar, kmer=12)
    sa = d_sa.cpu().numpy().view(np.uint32)
    del d_sa
    fm.set_tuning(block=64, refill=32, waves_per_cu=8)
    w = make_workload(5003, text, 1e7, 0.02, max_requests=200_000)
    # the same index over the other QuadRank layouts, counting every pattern directly
    by_layout = {}
    for name in ("16p", "32", "64", "24_8"):
        announce("serve-2^30 layout", name)
        other = qr.QuadFm(bwt, n + 1, dollar, kmer=12, layout=qr.LAYOUT_BY_NAME[name])
        by_layout[name] = other.count(to_dev(w.pat), to_dev(w.off)).cpu().numpy().view(np.uint32)
        other.check()
        other.free()
    del bwt
    torch.cuda.empty_cache()
    announce("serve-2^30 run", w.nreq, int(w.req_off[-1]))
    srv = NativeServer(fm, slots=4, budget_bytes=256 << 20, max_batch_patterns=1 << 18, check_free_memory=True)
    st = srv.run(w, deadline_s=120.0)
    assert srv.last_run_staged > 0  # pinned host arrays: batches staged by kernels
    assert not np.isnan(st.finish_s).any()
    assert np.all(st.finish_s >= w.arrival)
    npat = int(w.req_off[-1])
    served = srv.counts(0, npat)
    srv.free()
    announce("serve-2^30 direct")
    direct = fm.count(to_dev(w.pat), to_dev(w.off)).cpu().numpy().view(np.uint32)
    assert np.array_equal(served, direct)
    rng = np.random.default_rng(7)
    for r in rng.choice(w.nreq, min(20, w.nreq), replace=False):
        p0, p1 = int(w.req_off[r]), int(w.req_off[r + 1])
        pat = w.pat[int(w.off[p0]):int(w.off[p1])]
        off = (w.off[p0:p1 + 1] - w.off[p0]).astype(np.uint64)
        alone = fm.count(to_dev(pat), to_dev(off)).cpu().numpy().view(np.uint32)
        assert np.array_equal(served[p0:p1], alone)
    announce("serve-2^30 oracle: suffix-array check and every served count")
    sa = sa.astype(np.int64)
    assert oracle.check_sa(text, sa) == 0
    want_all = oracle.count_sa(text, sa, w.pat, w.off).astype(np.uint32)
    assert np.array_equal(served, want_all)
    for name, got in by_layout.items():
        assert np.array_equal(got, want_all), name
    del sa
    # oracle on sampled patterns (direct substring counting over the whole text)
    idx = np.sort(rng.choice(npat, 32, replace=False))
    pats = [w.pat[int(w.off[i]):int(w.off[i + 1])] for i in idx]
    s_off = np.zeros(len(pats) + 1, np.uint64)
    s_off[1:] = np.cumsum([p.size for p in pats])
    announce("serve-2^30 oracle sample")
    want = oracle.count_naive(text, np.concatenate(pats), s_off).astype(np.uint32)
    assert np.array_equal(served[idx], want)
    assert want.max() >= 1  # the sample holds patterns that occur
    fm.free()
