"""bench.py's command-line contract on the host: the single-GPU measurement
refuses a multi-GPU request with a message and exit code 2, before touching
any device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and "--gpus 2" in p.stderr
    assert p.stdout == ""


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_shares_add_up_to_the_whole_path():
    """The streaming kernels' shares of the algorithmic bytes are the terms of
    48T + 8V + 8P + 4Fh + 4: together exactly the whole path's bytes."""
    b = _bench()
    for nt, nv, p, fh in ((33554432, 16785409, 16040986, 65636404), (2048, 1089, 1024, 4096), (1, 3, 1, 3)):
        parts = [b.kernel_bytes(k, nt, nv, p, fh) for k in ("k_label", "k_relink", "k_compact")]
        assert sum(parts) == b.algorithmic_bytes(nt, nv, p, fh)
        assert b.kernel_bytes("k_relink", nt, nv, p, fh) == 36 * nt
        for k in ("k_repair", "k_fixup", "k_walk", "k_emit", "k_tile_scan"):
            assert b.kernel_bytes(k, nt, nv, p, fh) is None
        # the one-workgroup form of small meshes moves the whole path's bytes
        assert b.kernel_bytes("k_small", nt, nv, p, fh) == b.algorithmic_bytes(nt, nv, p, fh)


def test_cpu_baseline_reports_its_host():
    """The CPU baseline builds the oracle for this host, pins one core, says
    which, and restores the process's affinity afterwards."""
    import oracle
    from paper_2403_14723_amd import workloads as W
    b = _bench()
    before = os.sched_getaffinity(0)
    try:
        cpu, res = b.cpu_baseline(W.plain_small())
    finally:
        oracle.use_library(oracle._LIB)
    assert os.sched_getaffinity(0) == before
    assert cpu["cores"] == 1 and cpu["core"] in before and cpu["nproc"] >= 1
    assert cpu["cpu_model"] and "march=native" in cpu["compiler"]
    assert cpu["value"] > 0 and res.stats["npoly"] > 0


def test_every_workload_has_a_generator():
    """Each --workload name maps to a generator in the workloads module, and
    the Delaunay names carry their point counts."""
    b = _bench()
    from paper_2403_14723_amd import workloads as W
    for name, fn in b.WORKLOADS.items():
        assert callable(getattr(W, fn, None)), (name, fn)
    assert b.WORKLOADS["delaunay1000000_s21m"] == "delaunay_1m"
    assert b.WORKLOADS["delaunay4000000_s21m"] == "delaunay_4m"
