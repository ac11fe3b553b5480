"""Host logic of the profile records: which kernel a row's launch settings select, and which
rocprofv3 kernel names belong to which row (rank and prefix_rank share one sweep kernel)."""
from paper_2602_04103_amd import profiling as P


def test_launch_form():
    assert P.launch_form(None) == "pair"
    assert P.launch_form("default") == "pair"
    assert P.launch_form(dict(lanes=2, per_lane=1)) == "pair"
    assert P.launch_form(dict(lanes=1, per_lane=2)) == "lane"
    assert P.launch_form(dict(lanes=2, per_lane=2, sweep=1024)) == "sweep"
    assert P.launch_form(dict(lanes=2, sweep=0)) == "pair"
    assert P.traffic_key("quadrank_rank", 32, "sweep") == "quadrank_rank|L32|sweep"


def test_kernel_matches():
    rank_sweep = "void (anonymous namespace)::qr_sym_sweep_kernel<qr::QR32, 1, false, 4>(HIP_vector_type<unsigned int"
    pre_sweep = "void (anonymous namespace)::qr_sym_sweep_kernel<qr::QR32, 2, true, 8>(HIP_vector_type<unsigned int"
    pair = "void (anonymous namespace)::qr_rank1_pair_kernel<qr::QR16, 1>(HIP_vector_type<unsigned int, 4u>"
    lane = "void (anonymous namespace)::qr_rank1_kernel<qr::QR16, 1>(HIP_vector_type<unsigned int, 4u>"
    br = "void (anonymous namespace)::br_rank_sweep_kernel<qr::BR32, 2, 4>(HIP_vector_type<unsigned int"
    assert P.kernel_matches(rank_sweep, "quadrank_rank", "sweep", 32)
    assert not P.kernel_matches(rank_sweep, "quadrank_prefix_rank", "sweep", 32)
    assert P.kernel_matches(pre_sweep, "quadrank_prefix_rank", "sweep", 32)
    assert not P.kernel_matches(pre_sweep, "quadrank_rank", "sweep", 32)
    assert not P.kernel_matches(rank_sweep, "quadrank_rank", "sweep", 16)
    assert P.kernel_matches(pair, "quadrank_rank", "pair", 16)
    assert not P.kernel_matches(pair, "quadrank_rank", "lane", 16)  # qr_rank1_kernel is not a prefix of it
    assert P.kernel_matches(lane, "quadrank_rank", "lane", 16)
    assert not P.kernel_matches(lane, "quadrank_rank", "pair", 16)
    assert P.kernel_matches(br, "birank_rank_p0.5", "sweep", 32)
    assert not P.kernel_matches(br, "birank_rank_p0.5", "pair", 32)
    assert not P.kernel_matches(br, "quadrank_rank4", "sweep", 32)
    # named layouts: a 16-bit token does not match the paired or quarter-anchored variants
    paired = "void (anonymous namespace)::br_rank_sweep_kernel<qr::BR16P, 2, 4>(HIP_vector_type<unsigned int"
    quarter = "void (anonymous namespace)::br_rank_pair_kernel<qr::BR16X2, 1>(HIP_vector_type<unsigned int"
    multi = "void (anonymous namespace)::qr_rank4_pair_kernel<qr::QR24_8, 2>(HIP_vector_type<unsigned int"
    assert P.kernel_matches(paired, "birank_rank_p0.5", "sweep", "16p")
    assert not P.kernel_matches(paired, "birank_rank_p0.5", "sweep", 16)
    assert P.kernel_matches(quarter, "birank_rank_p0.05", "pair", "16x2")
    assert not P.kernel_matches(quarter, "birank_rank_p0.05", "pair", "16")
    assert P.kernel_matches(multi, "quadrank_rank4", "pair", "24_8")
    assert P.traffic_key("birank_rank_p0.5", "16p", "pair") == "birank_rank_p0.5|L16p|pair"


def test_traffic_records_match_the_current_sources():
    """Every committed HBM-traffic record was taken from the kernel sources as they stand (else the
    bench reports its traffic as null), and the measured bytes per query equal the algorithmic
    ones within 1 %."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles", "hbm_traffic.json")
    recs = json.load(open(path))["kernels"]
    algorithmic = {"quadrank_rank": 145, "quadrank_rank4": 168, "birank_rank_p0.5": 144, "birank_rank_p0.05": 144}
    assert set(k.split("|")[0] for k in recs) == set(algorithmic)
    for key, r in recs.items():
        assert r["source_hash"] == P.source_hash(r["sources"]), key
        per_query = r["hbm_bytes_per_launch"] / (1 << 24)
        assert abs(per_query / algorithmic[key.split("|")[0]] - 1) < 0.01, (key, per_query)
