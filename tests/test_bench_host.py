"""Host logic of bench.py (no GPU): the counter-measured traffic is reported
only for a summary taken on the current kernel sources at the same batch
size, and the flop model grows as its definition says."""
import os

import bench


def _tree(tmp_path, src_text, record):
    csrc = tmp_path / "paper_2504_10710_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text(src_text)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text("# summary\n\n" + record + "\n")
    return str(tmp_path)


def test_traffic_record_matches_sources_and_batch(tmp_path):
    root = str(tmp_path)
    os.makedirs(os.path.join(root, "paper_2504_10710_amd", "csrc"))
    with open(os.path.join(root, "paper_2504_10710_amd", "csrc", "k.hip"), "w") as f:
        f.write("kernel v1")
    dig = bench.sources_digest(root)
    os.makedirs(os.path.join(root, "profiles"))
    with open(os.path.join(root, "profiles", "k.md"), "w") as f:
        f.write(f"traffic-record: kernel=k<double, 128, 2>; batch=2048; sources={dig}; "
                f"bytes_per_launch=1234; fetch=1000; write=234\n")
    assert bench.measured_traffic("k<double, 128, 2>", 2048, root=root)[0] == 1234.0
    assert bench.measured_traffic("k<double, 128, 2>", 1024, root=root)[0] is None
    assert bench.measured_traffic("k<float, 128, 2>", 2048, root=root)[0] is None
    # a one-element record does not serve an element run of the same kernel
    assert bench.measured_traffic("k<double, 128, 2>", 2048, 4, root=root)[0] is None
    with open(os.path.join(root, "profiles", "k4.md"), "w") as f:
        f.write(f"traffic-record: kernel=k<double, 128, 2>; batch=2048; sources={dig}; "
                f"elements=4; bytes_per_launch=99; fetch=90; write=9\n")
    assert bench.measured_traffic("k<double, 128, 2>", 2048, 4, root=root)[0] == 99.0
    assert bench.measured_traffic("k<double, 128, 2>", 2048, root=root)[0] == 1234.0
    with open(os.path.join(root, "paper_2504_10710_amd", "csrc", "k.hip"), "w") as f:
        f.write("kernel v2")          # sources changed since the counters
    assert bench.measured_traffic("k<double, 128, 2>", 2048, root=root)[0] is None


def test_flop_model_monotone():
    a = bench.flops_per_solve(2, 128, 1, 1, 10, "fgmres", 30)
    b = bench.flops_per_solve(2, 128, 1, 1, 11, "fgmres", 30)
    c = bench.flops_per_solve(2, 128, 2, 1, 10, "fgmres", 30)
    assert 0 < a < b and a < c
    # one FGMRES iteration costs at least one cycle plus one fine operator
    n1 = 129
    apply_ = (4 * 2 * n1 + 7 + 1) * n1 ** 2
    assert b - a > apply_


def test_flop_model_collapsed_levels():
    """A collapsed level costs its matrix-vector product per visit and hides
    the levels below it: cheaper than the recursive count at gamma = 7."""
    full = bench.flops_per_solve(2, 128, 7, 1, 8, "fgmres", 30)
    coll = bench.flops_per_solve(2, 128, 7, 1, 8, "fgmres", 30, collapsed=(8, 16))
    assert 0 < coll < full
    one = bench.flops_per_solve(2, 128, 3, 1, 1, "fgmres", 30, collapsed=(16,))
    two = bench.flops_per_solve(2, 128, 3, 1, 1, "fgmres", 30, collapsed=(8, 16))
    assert one == two        # the p = 16 matrix hides p = 8


def test_element_flop_model():
    """Several elements: the per-visit operator count is the element
    contractions summed over elements (plus the assembly), the hierarchy
    stops at degree 2K with a dense exact solve, and K = 1 is unchanged."""
    import bench
    one = bench.flops_per_solve(2, 32, 2, 1, 10, "fgmres", 30)
    assert one == bench.flops_per_solve(2, 32, 2, 1, 10, "fgmres", 30, (), 1)
    K, p, gamma = 2, 16, 1
    # hand count: levels 16 and 8 (element degrees 8, 4), dense solve at degree 4
    def apply_(pl):
        ne1 = pl // K + 1
        return K * K * (8 * ne1 + 6) * ne1 ** 2 + (pl + 1) ** 2
    def transfer(pl):
        nb = K * (pl // K + 1) * (pl // (2 * K) + 1)
        return 2 * nb * (pl + 1 + pl // 2 + 1)
    sweeps = 2 * (1 + gamma)
    cycle = 0.0
    for depth, pl in enumerate((16, 8)):
        cycle += gamma ** depth * ((sweeps - 1 + gamma) * apply_(pl) + sweeps * 11 * (pl - 1) ** 2
                                   + 2 * gamma * transfer(pl))
    cycle += gamma ** 2 * 2 * (4 - 1) ** 4
    N = 17 ** 2
    iters = 3
    total = 0.0
    for j in range(iters):
        total += cycle + apply_(16) + 4 * (j + 1) * N + 3 * N
    total += 1 * (apply_(16) + 4 * N) + iters * 2 * N
    assert bench.flops_per_solve(2, p, gamma, 1, iters, "fgmres", 30, (), K) == total
