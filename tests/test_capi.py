"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol include/bgv.h declares, and the Python binding covers them."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bgv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bgv_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2604_19890_amd", "libbgv.so"))
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2604_19890_amd import bgv
    assert sorted(bgv.EXPORTED) == _declared()


def test_null_arguments_are_rejected_on_the_host():
    from paper_2604_19890_amd import bgv
    lib = bgv._lib
    assert lib.bgv_ctx_create(None, None, None) == 1  # BGV_E_ARG
    assert lib.bgv_sync(None) == 1
    assert lib.bgv_ct_words(None, 3) == 0
    assert lib.bgv_set_schedule(None, 0) == 1
    assert lib.bgv_set_ntt_split(None, 8) == 1


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asked for more it exits with status 2 and says so on its
    JSON line (before it touches the GPU)."""
    import json
    import subprocess
    import sys
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
