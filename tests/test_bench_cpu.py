"""Host-side logic of the benchmark: the M2P FLOP count of the implemented
recurrence and the gating of the recorded HBM traffic.  CPU only."""

import bench


def _m2p_count_by_terms(order):
    # the same count written term by term from the recurrence: per
    # coefficient k != 0, three sums over the first-lower neighbours
    # (a product each, an addition between consecutive ones), three over the
    # second-lower ones (additions only), then the combination; the
    # recurrence runs to degree P + 1 (the double layer's series); four
    # moment products and sums per coefficient of degree <= P, two of degree
    # P + 1; 14 for the pair set-up
    total = 14
    for s in range(order + 2):
        for i in range(s + 1):
            for j in range(s - i + 1):
                k = (i, j, s - i - j)
                total += (4 if s <= order else 2) * 2
                if s == 0:
                    continue
                first = [d for d in range(3) if k[d] >= 1]
                second = [d for d in range(3) if k[d] >= 2]
                total += 3 * (len(first) + (len(first) - 1))
                total += 3 * max(len(second) - 1, 0)
                if s == 1:
                    total += 1 + 1 + 3        # a = S1 iR2; by = ks Y1; ay = (Y1 + ks B1) iR2
                elif not second:
                    total += 2 + 1 + 4        # c1 S1 iR2; ks Y1; (c1 Y1 + ks B1) iR2
                else:
                    total += 4 + 2 + 7
    return total


def test_m2p_flops():
    assert bench._m2p_flops(4) == 1546
    assert bench._m2p_flops(5) == 2451
    for P in range(1, 8):
        assert bench._m2p_flops(P) == _m2p_count_by_terms(P)


def test_traffic_only_for_the_measured_case():
    for (mode, kernel, workload, precision), rec in bench.TRAFFIC.items():
        current = rec["sha"] == bench._sources_hash(bench.TRAFFIC_SOURCES[mode])
        t = bench.traffic_bytes(mode, kernel, workload, precision)
        # recorded counters hold only while the kernel's sources are unchanged
        if current:
            assert t is not None and 1e8 < t < 3e8
        else:
            assert t is None
        assert bench.traffic_bytes(mode, kernel, "sphere_81920", precision) is None
        assert bench.traffic_bytes(mode, kernel, workload, "fp64") is None
    assert bench.traffic_bytes("direct", "p2p", "globule_5000", "mixed") is None
