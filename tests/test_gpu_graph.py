"""HIP graph capture of the query and count launch sequences: every replay (with eager work and
synchronisations in between) must reproduce the eager results exactly."""
import numpy as np
import pytest
import torch

import datagen
from tests.gpu_util import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def test_graph_replays_rank_rank4_and_counts():
    qr = require_gpu()
    n = 2 * 61440 + 777
    codes = datagen.dna_codes(61, n)
    h = qr.QuadRank(to_dev(datagen.pack2(codes)), n)
    q = to_dev(datagen.queries(62, n, 300_000))
    c = to_dev(datagen.symbols(63, 300_000))
    fm = qr.QuadFm.from_text(codes[:50_000])
    pat, off, _ = datagen.patterns(64, codes[:50_000], 20_000)
    dp, do = to_dev(pat), to_dev(off)
    bits = datagen.bits(65, 400_000)
    br = qr.BiRank(to_dev(bits), 400_000)
    qb = to_dev(datagen.queries(66, 400_000, 100_000))

    # eager reference
    e1 = h.rank(q, c).clone()
    e4 = h.rank4(q).clone()
    ef = fm.count(dp, do).clone()
    eb = fm.count_batched(dp, do, 1024).clone()
    er = br.rank(qb).clone()
    torch.cuda.synchronize()

    s = torch.cuda.Stream()
    o1 = torch.empty_like(e1)
    o4 = torch.empty_like(e4)
    of = torch.empty_like(ef)
    ob = torch.empty_like(eb)
    orr = torch.empty_like(er)
    announce("graph capture")
    with torch.cuda.stream(s):
        g = qr.Graph(s)
        with g:
            h.rank(q, c, o1, stream=s)
            h.rank4(q, o4, stream=s)
            fm.count(dp, do, of, stream=s)
            fm.count_batched(dp, do, 1024, ob, stream=s)
            br.rank(qb, orr, stream=s)
    for rep in range(3):
        for t in (o1, o4, of, ob, orr):
            t.fill_(-1)                         # eager work between replays
        torch.cuda.synchronize()
        announce("graph replay", rep)
        g.launch(s)
        s.synchronize()
        assert torch.equal(o1, e1) and torch.equal(o4, e4)
        assert torch.equal(of, ef) and torch.equal(ob, eb) and torch.equal(orr, er)
    g.free()


def test_graph_replays_prefix_rank_intervals_and_locate():
    """prefix_rank on the 32-bit layout and the whole locate pipeline (intervals, output offsets, LF
    walks; the number of positions taken from an eager run) captured in one graph."""
    qr = require_gpu()
    n = 3 * 57344 + 99
    codes = datagen.dna_codes(71, n)
    h = qr.QuadRank(to_dev(datagen.pack2(codes)), n, layout=qr.QR_LAYOUT_32)
    q = to_dev(datagen.queries(72, n, 200_000))
    c = to_dev(datagen.symbols(73, 200_000))
    text = codes[:60_000].copy()
    datagen.plant_repeats(74, text, nseg=5, seglen=1000, copies=6, sub=0.01)
    fm = qr.QuadFm.from_text(text, locate_rate=8, device_sa=True)
    pat, off, _ = datagen.patterns(75, text, 5000, minlen=8, maxlen=40)
    dp, do = to_dev(pat), to_dev(off)
    npat = off.size - 1

    ep = h.prefix_rank(q, c).clone()
    eiv = fm.intervals(dp, do).clone()
    est = torch.empty(npat + 1, dtype=torch.int64, device="cuda")
    qr.quadfm_locate_offsets(fm.h, eiv, est)
    total = int(est[npat].item())
    epos = torch.empty(total, dtype=torch.int32, device="cuda")
    qr.quadfm_locate(fm.h, eiv, est, total, epos)
    fm.check()
    assert total > npat // 2

    s = torch.cuda.Stream()
    op, oiv = torch.empty_like(ep), torch.empty_like(eiv)
    ost, opos = torch.empty_like(est), torch.empty_like(epos)
    announce("graph capture locate", total)
    with torch.cuda.stream(s):
        g = qr.Graph(s)
        with g:
            h.prefix_rank(q, c, op, stream=s)
            fm.intervals(dp, do, oiv, stream=s)
            qr.quadfm_locate_offsets(fm.h, oiv, ost, stream=s)
            qr.quadfm_locate(fm.h, oiv, ost, total, opos, stream=s)
    for rep in range(3):
        for t in (op, oiv, ost, opos):
            t.fill_(-1)
        torch.cuda.synchronize()
        announce("graph replay locate", rep)
        g.launch(s)
        s.synchronize()
        assert torch.equal(op, ep) and torch.equal(oiv, eiv)
        assert torch.equal(ost, est) and torch.equal(opos, epos)
    fm.check()
    g.free()


def test_graph_replays_sweep_form():
    """The position-ordered (sweep) launches of rank, prefix_rank, rank4 and BiRank rank, captured
    with the tile sizes the tuner offers, replayed three times."""
    qr = require_gpu()
    n = 3 * 57344 + 5
    codes = datagen.dna_codes(81, n)
    h = qr.QuadRank(to_dev(datagen.pack2(codes)), n, layout=qr.QR_LAYOUT_32)
    q = to_dev(datagen.queries(82, n, 250_001))
    c = to_dev(datagen.symbols(83, 250_001))
    br = qr.BiRank(to_dev(datagen.bits(84, 500_000)), 500_000, layout=qr.QR_LAYOUT_32)
    qb = to_dev(datagen.queries(85, 500_000, 120_007))
    h.set_tuning(lanes=2, per_lane=1, sweep=1024)
    br.set_tuning(lanes=2, per_lane=2, sweep=4096)
    e1, ep, e4, eb = h.rank(q, c).clone(), h.prefix_rank(q, c).clone(), h.rank4(q).clone(), br.rank(qb).clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    o1, op, o4, ob = (torch.empty_like(t) for t in (e1, ep, e4, eb))
    announce("graph capture sweep")
    with torch.cuda.stream(s):
        g = qr.Graph(s)
        with g:
            h.rank(q, c, o1, stream=s)
            h.prefix_rank(q, c, op, stream=s)
            h.rank4(q, o4, stream=s)
            br.rank(qb, ob, stream=s)
    for rep in range(3):
        for t in (o1, op, o4, ob):
            t.fill_(-1)
        torch.cuda.synchronize()
        announce("graph replay sweep", rep)
        g.launch(s)
        s.synchronize()
        assert torch.equal(o1, e1) and torch.equal(op, ep) and torch.equal(o4, e4) and torch.equal(ob, eb)
    g.free()
