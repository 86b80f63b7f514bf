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
