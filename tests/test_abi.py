"""Host-only checks of the C ABI: the library loads, exports every function
include/lks.h declares, and validates problems without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2608_01071_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lks_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2608_01071_amd import lks
    return lks.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/lks.h but not exported"


def test_library_matches_its_sources(L):
    """The build embeds the SHA-256 of the sources; the loaded library's
    equals the digest of the sources next to it."""
    from paper_2608_01071_amd.srcdigest import source_digest
    want = source_digest()
    assert want is not None and len(want) == 64
    assert L.lks_source_digest().decode() == want


def declared_parameter_counts():
    src = open(os.path.join(ROOT, "include", "lks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(lks_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", src):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_declares_every_argument_type(L):
    """Every entry point the header declares has its argument types declared
    in the binding, one per parameter: without them ctypes passes Python
    ints as 32-bit C ints and truncates device pointers."""
    counts = declared_parameter_counts()
    assert set(counts) == set(declared_functions())
    for name, n in counts.items():
        at = getattr(L, name).argtypes
        if n == 0:
            continue
        assert at is not None, f"{name}: no argtypes in the binding"
        assert len(at) == n, f"{name}: {len(at)} argtypes for {n} parameters"


def test_plan_validation_and_workspace(L):
    from paper_2608_01071_amd import lks
    p, *_ = W.c1()
    h = C.c_void_p()
    nb = C.c_size_t()
    s = lks.to_struct(p)
    assert L.lks_plan_create(C.byref(s), C.byref(h), C.byref(nb)) == 0
    assert nb.value > 0 and nb.value % 256 == 0
    # checkpoint storage grows as K shrinks
    s2 = lks.to_struct(p.replace(ckpt_k=10))
    h2 = C.c_void_p()
    nb2 = C.c_size_t()
    assert L.lks_plan_create(C.byref(s2), C.byref(h2), C.byref(nb2)) == 0
    assert nb2.value != nb.value
    L.lks_plan_destroy(h)
    L.lks_plan_destroy(h2)
    # the ALKS scheme carries the raw first-moment part of the adjoint
    # velocity in two more [d][N] slots
    s5 = lks.to_struct(p.replace(scheme=1))
    h5 = C.c_void_p()
    nb5 = C.c_size_t()
    assert L.lks_plan_create(C.byref(s5), C.byref(h5), C.byref(nb5)) == 0
    assert nb5.value >= nb.value + 2 * p.d * p.N * 8
    L.lks_plan_destroy(h5)
    # J2 keeps per-block step sums and a seed slot on the body box
    s6 = lks.to_struct(p.replace(objective=1, w_d=0.1, w_t=0.2, l_m=3.0))
    h6 = C.c_void_p()
    nb6 = C.c_size_t()
    assert L.lks_plan_create(C.byref(s6), C.byref(h6), C.byref(nb6)) == 0
    assert nb6.value > nb.value
    L.lks_plan_destroy(h6)
    po, *_ = W.oar(nt=20)
    assert po.objective == 1 and po.xg_min[0] == po.xg_max[0]
    assert L.lks_plan_create(C.byref(lks.to_struct(po)), C.byref(h6), C.byref(nb6)) == 0
    L.lks_plan_destroy(h6)
    bad = [p.replace(d=4), p.replace(n=(64, 3, 1)), p.replace(nt=0), p.replace(r_t=0),
           p.replace(ckpt_k=500), p.replace(precision=2), p.replace(q=0.0),
           p.replace(scheme=2), p.replace(scheme=-1), p.replace(objective=2),
           p.replace(objective=1, w_d=0.1, w_t=0.1, l_m=0.0)]
    p3, *_ = W.make_3d(16, 4, 5, 2, nu=0.1, seed=0)
    p3 = p3.replace(ckpt_k=5)
    h0 = C.c_void_p()
    assert L.lks_plan_create(C.byref(lks.to_struct(p3)), C.byref(h0), C.byref(nb)) == 0
    L.lks_plan_destroy(h0)
    bad.append(p3.replace(bc=(1, 1, 1)))
    bad.append(p3.replace(objective=1, l_m=2.0))  # J2 is 2D only
    # 3D (p, u) states of 4 GiB and more (2^28 nodes in FP32, 2^27 in FP64)
    bad.append(p3.replace(n=(512, 512, 1024), precision=0))
    bad.append(p3.replace(n=(512, 512, 512), precision=1))
    for b in bad:
        h3 = C.c_void_p()
        rc = L.lks_plan_create(C.byref(lks.to_struct(b)), C.byref(h3), C.byref(nb))
        assert rc == lks.LKS_EINVAL, b
        assert len(L.lks_last_error()) > 0
    # just below: 2^28 - 2^18 nodes in FP32, 2^27 - 2^18 in FP64
    for n, prec in (((512, 512, 1023), 0), ((512, 512, 511), 1)):
        h4 = C.c_void_p()
        assert L.lks_plan_create(C.byref(lks.to_struct(p3.replace(n=n, precision=prec))),
                                 C.byref(h4), C.byref(nb)) == 0, n
        L.lks_plan_destroy(h4)


def test_null_arguments_rejected_before_any_launch(L):
    from paper_2608_01071_amd import lks
    p, *_ = W.c1()
    h = C.c_void_p()
    nb = C.c_size_t()
    assert L.lks_plan_create(C.byref(lks.to_struct(p)), C.byref(h), C.byref(nb)) == 0
    assert L.lks_forward(h, None, None, None, None, None, None, None, None) == lks.LKS_EINVAL
    assert L.lks_adjoint(h, *([None] * 11)) == lks.LKS_EINVAL
    one = C.c_double(1.0)
    assert L.lks_design_filter(h, None, one, one, C.c_double(0.5), None, None) == lks.LKS_EINVAL
    assert L.lks_design_filter_adjoint(h, None, one, one, C.c_double(0.5), None, None, None,
                                       None) == lks.LKS_EINVAL
    assert L.lks_constraints(h, None, None, None, None, one, one, one, None, None, None, None,
                             None) == lks.LKS_EINVAL
    assert L.lks_step(h, None, None, None, None, None) == lks.LKS_EINVAL
    L.lks_plan_destroy(h)


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on exactly one GPU: --gpus N > 1 exits with a message
    (before touching a device)."""
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr



def test_bench_traffic_is_read_only_for_its_kernel_source(tmp_path, monkeypatch):
    """The roofline's measured HBM traffic comes from the committed counter
    summary only while the digest that summary names is the kernel source's;
    after any change to the source (or without a summary) it is None, and the
    bench line reports it as null."""
    import hashlib
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "kernels.hip"
    src.write_bytes(b"kernel source, first form")
    digest = hashlib.sha256(b"kernel source, first form").hexdigest()
    summary = tmp_path / "traffic.txt"
    summary.write_text("# counter summary\n"
                       f"kernel_source_sha256 {digest}\n"
                       "traffic k_fwd3d<float> 123\n"
                       "traffic k_adj3d<float> 456\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(summary))
    assert bench.measured_traffic("fwd_step") == 123.0
    assert bench.measured_traffic("adj_step") == 456.0
    src.write_bytes(b"kernel source, second form")
    assert bench.measured_traffic("fwd_step") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.txt"))
    assert bench.measured_traffic("fwd_step") is None

def test_noalloc_entry_point_rejects_oversized_design_grid(L):
    """The allocation-free chain rule refuses, on the host and before any
    device call, a plan with more inner design points than its fixed
    scratch holds."""
    from paper_2608_01071_amd import lks
    p = W.Problem(d=3, n=(200, 200, 200), bc=(1, 1, 0), m=(130, 130, 130), margin=4,
                  xg_min=(100.0, 100.0, 100.0), xg_max=(100.0, 100.0, 100.0),
                  tgt_lo=(0, 0, 0), tgt_hi=(1, 1, 1), nt=4, r_t=1, r_w=1, precision=0)
    assert p.M > (1 << 21)
    h = C.c_void_p()
    nb = C.c_size_t()
    assert L.lks_plan_create(C.byref(lks.to_struct(p)), C.byref(h), C.byref(nb)) == 0
    dummy = C.c_void_p(256)  # never dereferenced: the size check comes first
    rc = L.lks_design_filter_adjoint_noalloc(h, dummy, C.c_double(2.0), C.c_double(0.0),
                                            C.c_double(0.5), dummy, dummy, None)
    assert rc == lks.LKS_EINVAL
    assert b"exceed its scratch" in L.lks_last_error()
    L.lks_plan_destroy(h)
