"""bench.py's command-line contract that needs no GPU: it runs on one GPU and
refuses a multi-GPU request with a message instead of starting."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1",
                          "--warmup", "0"], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode != 0
    msg = out.stdout + out.stderr
    assert "one GPU" in msg and "--gpus 2" in msg, msg
