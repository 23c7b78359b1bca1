"""The oracle's operation-counting scalar against hand counts of its plain
formulation, and the algorithmic flop counts of bench.py's roofline against
it (CPU only): the count used for a reconstruction never exceeds what the
plain formulation needs."""
import importlib.util
import os

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def bench_module():
    spec = importlib.util.spec_from_file_location("bench_counts", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def total(c):
    return sum(c.values())


def test_counts_of_the_plain_formulation():
    # WENO7-Z by hand: candidates 4 x (4 mul, 3 add, 1 div) = 32; smoothness
    # 4 x 23 = 92; tau 2 mul + 3 add = 5; tau/(b + eps) 4 x 2 = 8; squares 4 x 2
    # = 8 (the power loop starts from 1); alpha 4 x 2 = 8; sum 3; combination
    # 4 x 3 = 12: 168.  Jiang-Shu: (eps + b)^2 and d/() 4 x 4 = 16 instead of
    # tau, ratios, squares and alpha (29): 155.  Linear: candidates 32 + 4 mul
    # + 3 add = 39.
    assert total(O.count_flops("weno7", "z")) == 168
    assert total(O.count_flops("weno7", "js")) == 155
    assert total(O.count_flops("weno7", "linear")) == 39
    assert O.count_flops("weno7", "z")["sqrt"] == 0
    # recovery: two square roots (the closed form and n = N sqrt(1 - v^2))
    c = O.count_flops("c2p")
    assert c["sqrt"] == 2 and total(c) == 28


def test_roofline_counts_do_not_exceed_the_plain_formulation():
    b = bench_module()
    plain = {"z": ("weno7", "z"), "js": ("weno7", "js"), "linear": ("weno7", "linear"),
             "z5": ("weno5", "z"), "js5": ("weno5", "js"), "linear5": ("weno5", "linear")}
    for scheme, (w, s) in plain.items():
        assert b.RECON_FLOPS[scheme] <= total(O.count_flops(w, s)), scheme
    assert b.FLOPS_PER_CELL_UPDATE <= 30 * total(O.count_flops("weno7", "z")) + total(O.count_flops("c2p")) + 3 * 35 + 15
