"""The C ABI library loads on a machine without a GPU and exports every
function include/rwmi.h declares; host-only entry points work there."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "rwmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(rwmi_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    d = declared()
    for name in ("rwmi_create_domain", "rwmi_add_metaball_particle", "rwmi_seed_walkers", "rwmi_step",
                 "rwmi_read_moments", "rwmi_batch_step", "rwmi_footprint_bytes"):
        assert name in d


def test_library_exports_every_declared_symbol():
    from paper_2308_05007_amd import binding as B
    L = B.lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding knows the whole surface
    assert set(declared()) == set(B.SIGNATURES), set(declared()) ^ set(B.SIGNATURES)


def test_footprint_is_host_only_and_monotone():
    from paper_2308_05007_amd import binding as B
    from paper_2308_05007_amd import workloads as W
    dom = W.config_channel(precision="fp32")["domain"]
    a = B.footprint_bytes(dom, 20, 240, 1_000_000)
    b = B.footprint_bytes(dom, 20, 240, 2_000_000)
    c = B.footprint_bytes(dict(dom, precision="fp16"), 20, 240, 1_000_000)
    assert 0 < c < a < b
    # distributions dominate: at 128^3 FP32 (160 MB) one lattice streamed in
    # place; at 256^3 (1.27 GB) two lattices
    assert 19 * 4 * 128 ** 3 < a < 2 * 19 * 4 * 128 ** 3
    big = B.footprint_bytes(dict(dom, n=(256, 256, 256)), 20, 240, 1_000_000)
    assert big > 2 * 19 * 4 * 256 ** 3


def test_errors_without_a_gpu_are_reported_not_raised_by_the_library():
    from paper_2308_05007_amd import binding as B
    L = B.lib()
    st = L.rwmi_step(None, 1)
    assert st == B.RWMI_EINVAL
    assert L.rwmi_last_error(None)


@pytest.mark.parametrize("change,what", [
    (dict(tau=0.5), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(n=(0, 8, 8)), "n[0]"),
    (dict(n=(8, 2, 8), bc=("periodic", "wall", "periodic")), "wall axis"),
    (dict(n=(2048, 1024, 1024)), "too large"),
    (dict(D=-1.0), "diffusivity"),
])
def test_invalid_domains_are_rejected_before_the_device(change, what):
    """Descriptor checks run on the host first, so they report EINVAL (and
    no domain) on a machine without a GPU; 2^31 nodes is one past the
    largest lattice the 32-bit node indices allow."""
    import ctypes as C
    from paper_2308_05007_amd import binding as B
    from paper_2308_05007_amd import workloads as W
    dom = dict(W.config_channel(precision="fp32")["domain"], **change)
    d = B.make_desc(dom)
    h = C.c_void_p(1)
    assert B.lib().rwmi_create_domain(C.byref(d), C.byref(h)) == B.RWMI_EINVAL
    assert not h.value
    assert what in B.lib().rwmi_last_error(None).decode()


def test_invalid_precision_and_callback_pairs_are_rejected():
    import ctypes as C
    from paper_2308_05007_amd import binding as B
    from paper_2308_05007_amd import workloads as W
    d = B.make_desc(W.config_channel(precision="fp32")["domain"])
    d.precision = 99
    h = C.c_void_p()
    assert B.lib().rwmi_create_domain(C.byref(d), C.byref(h)) == B.RWMI_EINVAL
    d = B.make_desc(W.config_channel(precision="fp32")["domain"])
    d.alloc = B.ALLOC_FN(lambda n, ctx: None)
    assert B.lib().rwmi_create_domain(C.byref(d), C.byref(h)) == B.RWMI_EINVAL
    assert "together" in B.lib().rwmi_last_error(None).decode()


def test_stream_probe_rejects_bad_arguments_before_any_launch():
    import ctypes as C
    from paper_2308_05007_amd import binding as B
    L = B.lib()
    buf = C.c_void_p(16)  # never dereferenced: every case fails its checks first
    for streams, elem, n, src in ((3, 4, 256, buf), (19, 4, 300, buf), (19, 2, 0, buf), (4, 4, 1 << 32, buf),
                                  (4, 4, 256, None), (4, 8, 256, buf), (4, 1, 256, buf)):
        assert L.rwmi_stream_probe(streams, elem, 1, n, src, buf, None) == B.RWMI_EINVAL
    assert L.rwmi_stream_probe(5, 4, 0, 256, buf, buf, None) == B.RWMI_EINVAL
    assert "streams" in L.rwmi_last_error(None).decode()
    assert L.rwmi_stream_probe(4, 3, 0, 256, buf, buf, None) == B.RWMI_EINVAL
    assert "elem_bytes" in L.rwmi_last_error(None).decode()


def build_c_client(out_dir):
    """Compile tests/helpers/abi_client.c, a client of the ABI in plain C99
    (no Python, no PyTorch), against include/rwmi.h and librwmi.so."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    pkg = os.path.join(ROOT, "paper_2308_05007_amd")
    exe = os.path.join(str(out_dir), "abi_client")
    subprocess.check_call([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "helpers", "abi_client.c"),
                           "-L" + pkg, "-lrwmi", "-Wl,-rpath," + pkg, "-o", exe])
    return exe


def test_header_is_c99_and_a_c_client_links(tmp_path):
    from paper_2308_05007_amd import binding as B
    B.lib()  # the library is built
    exe = build_c_client(tmp_path)
    assert os.access(exe, os.X_OK)
