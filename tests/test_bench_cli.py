"""Host-side checks of the benchmark script (no GPU): the one-GPU guard
and the source digest that keys its stored HBM-traffic figures."""
import io
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_digest_covers_every_kernel_source(monkeypatch):
    """The digest changes when any kernel source file or the code generator
    changes, so stored counter figures go stale (and are reported as null)
    with any kernel edit."""
    sys.path.insert(0, ROOT)
    import bench
    import glob
    csrc = os.path.join(ROOT, "paper_2506_02602_amd", "csrc")
    # every source file; generated/ holds the code generator's output
    srcs = sorted(f for f in glob.glob(os.path.join(csrc, "*")) if os.path.isfile(f))
    assert srcs and all(f.endswith((".hip", ".h")) for f in srcs)
    d0 = bench.kernel_digest()
    assert d0 == bench.kernel_digest() and len(d0) == 16
    real_open = open
    for f in srcs + [os.path.join(ROOT, "paper_2506_02602_amd", "codegen.py")]:
        def patched(path, mode="r", *a, _f=f, **k):
            fh = real_open(path, mode, *a, **k)
            if os.path.abspath(path) == _f and "b" in mode:
                data = fh.read() + b" "
                fh.close()
                return io.BytesIO(data)
            return fh
        monkeypatch.setattr("builtins.open", patched)
        assert bench.kernel_digest() != d0, os.path.basename(f)
        monkeypatch.setattr("builtins.open", real_open)
