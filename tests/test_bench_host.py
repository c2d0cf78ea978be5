"""Host-side checks of bench.py's command line: more than one GPU is refused
with a message (the FMM here runs on one GPU), before anything touches a GPU."""
import os
import subprocess
import sys


def test_multi_gpu_request_is_refused(repo_root):
    for n in ("2", "8"):
        r = subprocess.run([sys.executable, os.path.join(repo_root, "bench.py"), "--gpus", n],
                           capture_output=True, text=True, timeout=120, cwd=repo_root)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""
