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
    assert bench.measured_traffic("k<double, 128, 2>", 2048, root)[0] == 1234.0
    assert bench.measured_traffic("k<double, 128, 2>", 1024, root)[0] is None
    assert bench.measured_traffic("k<float, 128, 2>", 2048, root)[0] is None
    with open(os.path.join(root, "paper_2504_10710_amd", "csrc", "k.hip"), "w") as f:
        f.write("kernel v2")          # sources changed since the counters
    assert bench.measured_traffic("k<double, 128, 2>", 2048, root)[0] is None


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
