"""Host-side parts of the benchmark that need no GPU: the one-GPU guard and
the readers of the committed counter summaries."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The benchmark measures one GPU: --gpus 2 exits with status 2 and says
    why, before anything touches a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_too_few_steps_are_refused():
    """Fewer timed steps than one launch of the four-step kernel would leave
    no launch to time: refused with status 2 before any device work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "--steps" in r.stderr and not r.stdout.strip()


def test_summary_readers_take_only_profiled_shapes():
    """Counter figures are reported only for launch shapes that the
    committed summaries cover; any other shape reads as None (null in the
    JSON line), never as another shape's figures."""
    assert bench.valu_issue(dict(kernel=3, block=256, rows=0)) is None
    assert bench.valu_issue(dict(kernel=4, block=512, rows=8)) is None
    assert bench.counter_traffic(dict(kernel=4, block=1024, rows=0)) is None
    a = bench.valu_issue(dict(kernel=4, block=128, rows=0))
    b = bench.valu_issue(dict(kernel=4, block=256, rows=0))
    assert a is not None and b is not None and a != b
