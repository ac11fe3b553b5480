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
