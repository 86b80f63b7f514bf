"""The committed rocprofv3 summaries describe the kernels as they are: each
names the hash of the sources it measured, and that hash must still match.
bench.py reads two of them (HBM traffic, VALU issue) only while it matches;
this test makes a kernel change without new profiles fail loudly instead."""
import glob
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HASH_LINE = re.compile(r"^(\w+)_kernel_sources_sha256_16: ([0-9a-f]{16})", re.M)


def summaries():
    return sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))


def test_every_summary_names_its_sources():
    assert summaries(), "no profile summaries committed"
    for path in summaries():
        text = open(path).read()
        assert HASH_LINE.search(text), path
        assert "rocprofv3" in text, path


def test_summaries_match_current_kernel_sources():
    for path in summaries():
        for family, digest in HASH_LINE.findall(open(path).read()):
            assert family in bench.KERNEL_SOURCES, (path, family)
            assert bench.kernel_hash(family) == digest, (
                "%s was taken on other %s kernel sources" % (os.path.basename(path), family))


def test_summaries_give_commands_on_committed_files():
    """Every command line names only the repository's own programs."""
    for path in summaries():
        for line in open(path):
            if "rocprofv3 " in line and " -- " in line:
                prog = line.split(" -- ", 1)[1].split()
                assert prog[0] in ("python3", "python"), (path, line)
                assert prog[1].startswith("$REPO/") and "_work" not in prog[1], (path, line)
                assert os.path.exists(os.path.join(ROOT, prog[1][len("$REPO/"):])), (path, line)


def test_bench_reads_traffic_and_issue_for_the_headline_shapes():
    """The four-step shapes the autotuner picks for the 4096^2 workload
    (block 256 with fitted rows on a developed field, block 128 within 3%)
    have HBM traffic and VALU issue figures in the committed counters, so
    the benchmark line reports them rather than null."""
    for block in (128, 256):
        t = bench.counter_traffic(dict(kernel=4, block=block, rows=0))
        assert t is not None and 1.0 < t / (18 * 4 * 4096 * 4096) < 1.2, (block, t)
        v = bench.valu_issue(dict(kernel=4, block=block, rows=0))
        assert v is not None and 0 < v["valu_issue_busy"] <= 1, block
        assert v["lane_instructions_per_update"] > 100, block
    for storage in ("f32", "f64", "f16"):
        assert bench.counter_traffic3(storage) is not None, storage
