"""Concurrent queries on one handle from several streams (the C ABI allows it: the structures are
read-only; FM counts take caller-owned queue heads): every result must equal the eager result of
the same call run alone, and the oracle's."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev, to_host_u64

pytestmark = pytest.mark.gpu


def test_rank_calls_overlap_on_streams():
    qr = require_gpu()
    n = 9 * 57344 + 31
    codes = datagen.dna_codes(91, n)
    packed = datagen.pack2(codes)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_32)
    nb = 3 * 64512 * 16 + 7
    bits = datagen.bits(92, nb)
    br = qr.BiRank(to_dev(bits), nb)
    streams = [torch.cuda.Stream() for _ in range(4)]
    qs = [datagen.queries(93 + k, n, 400_000 + k) for k in range(4)]
    cs = [datagen.symbols(97 + k, 400_000 + k) for k in range(4)]
    qb = [datagen.queries(101 + k, nb, 300_000 + k) for k in range(4)]
    dq, dc, dqb = [to_dev(x) for x in qs], [to_dev(x) for x in cs], [to_dev(x) for x in qb]
    outs = []
    torch.cuda.synchronize()
    announce("concurrent rank streams")
    for rep in range(3):
        outs = []
        for k, s in enumerate(streams):
            with torch.cuda.stream(s):
                if k == 1:
                    h.set_tuning(lanes=2, per_lane=1, sweep=2048)  # handle settings are read at launch
                o1 = h.rank(dq[k], dc[k], stream=s)
                o4 = h.rank4(dq[k], stream=s)
                op = h.prefix_rank(dq[k], dc[k], stream=s)
                ob = br.rank(dqb[k], stream=s)
                outs.append((o1, o4, op, ob))
                if k == 1:
                    h.set_tuning(lanes=2, per_lane=1)
        torch.cuda.synchronize()
    h.check()
    br.check()
    for k in range(4):
        o1, o4, op, ob = outs[k]
        assert np.array_equal(to_host_u64(o1), oracle.rank_dna(packed, n, qs[k], cs[k]))
        assert np.array_equal(to_host_u64(o4).reshape(-1, 4), oracle.rank4_dna(packed, n, qs[k]))
        assert np.array_equal(to_host_u64(op), oracle.prefix_rank_dna(packed, n, qs[k], cs[k]))
        assert np.array_equal(to_host_u64(ob), oracle.rank_bits(bits, nb, qb[k]))


def test_fm_counts_with_own_queue_heads_overlap():
    qr = require_gpu()
    n = 300_000
    text = datagen.dna_codes(111, n)
    datagen.plant_repeats(112, text, nseg=10, seglen=2000, copies=8, sub=0.01)
    fm = qr.QuadFm.from_text(text)
    sa = oracle.suffix_array(text)
    streams = [torch.cuda.Stream() for _ in range(4)]
    sets = [datagen.patterns(113 + k, text, 30_000 + 1000 * k) for k in range(4)]
    want = [oracle.count_sa(text, sa, p, o).astype(np.uint32) for p, o, _ in sets]
    dev = [(to_dev(p), to_dev(o)) for p, o, _ in sets]
    heads = [torch.empty(1, dtype=torch.int64, device="cuda") for _ in range(4)]
    announce("concurrent fm streams")
    for rep in range(3):
        outs = []
        for k, s in enumerate(streams):
            dp, do = dev[k]
            out = torch.empty(do.numel() - 1, dtype=torch.int32, device="cuda")
            with torch.cuda.stream(s):
                qr.quadfm_count_ws(fm.h, dp, do, out, heads[k], stream=s)
            outs.append(out)
        torch.cuda.synchronize()
        fm.check()
        for k in range(4):
            assert np.array_equal(outs[k].cpu().numpy().view(np.uint32), want[k]), (rep, k)
