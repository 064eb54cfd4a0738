"""C ABI of libdq: loads without a GPU, exports every symbol include/*.h
declare, and validates parameters on the host (no compute calls)."""

import ctypes as C
import os
import re

import numpy as np

import pytest

from paper_2201_04614_amd import binding as dq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(dq.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return dq.lib()


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        with open(os.path.join(ROOT, "include", h)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(dq_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_lists_every_export():
    from paper_2201_04614_amd import batch as BT
    from paper_2201_04614_amd import huffman as HF
    from paper_2201_04614_amd import mixed as MX
    from paper_2201_04614_amd import selector as SEL
    assert declared_functions() == sorted(dq.EXPORTS + SEL.EXPORTS + BT.EXPORTS + HF.EXPORTS + MX.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_strerror(L):
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert dq.strerror(st) and "unknown" not in dq.strerror(st)
    assert "unknown" in dq.strerror(42)


def test_validate_host_only(L):
    ok = dq.make_params((10, 10), 1e-3, "abs", 4, "zero", 512)
    assert dq.validate(ok) == dq.DQ_OK
    bad = [dict(shape=(0, 10)), dict(eb=0.0), dict(eb=float("nan")), dict(eb=1e-320),
           dict(block=0), dict(pad=9), dict(pad=-1), dict(radius=0), dict(radius=32769), dict(eb_mode=3),
           dict(shape=(65536, 65536))]
    base = dict(shape=(10, 10), eb=1e-3, eb_mode="abs", block=4, pad="zero", radius=512)
    for b in bad:
        kw = dict(base)
        kw.update(b)
        assert dq.validate(dq.make_params(**kw)) == dq.DQ_EINVAL, b
    p = dq.make_params((1, 1, 1), 1.0)
    p.ndim = 4
    assert dq.validate(p) == dq.DQ_EINVAL
    # valid for the method, outside the GPU kernels' coverage
    for shape, B in (((100,), 6), ((100,), 8192), ((64, 64), 512), ((8, 8, 8), 128), ((436, 207), 128),
                     ((10, 66), 256)):
        assert dq.validate(dq.make_params(shape, 1e-3, "abs", B)) == dq.DQ_ENOTSUP
    for shape, B in (((100,), 4096), ((64, 64), 256), ((8, 8, 8), 64), ((5, 7, 9), 1), ((207, 436), 128),
                     ((3, 68), 256), ((436, 207), 64)):
        assert dq.validate(dq.make_params(shape, 1e-3, "abs", B)) == dq.DQ_OK


def test_counts_and_workspace(L):
    p = dq.make_params((20, 33, 17), 1e-3, "rel", 8, "edge_mean", 512)
    nb = 3 * 5 * 3
    assert dq.num_blocks(p) == nb
    assert dq.pad_count(p) == nb * 3
    for pad, n in (("zero", 0), ("block_mean", nb), ("global_mean", 1), ("block_min", nb), ("block_max", nb),
                   ("global_min", 1), ("global_max", 1)):
        assert dq.pad_count(dq.make_params((20, 33, 17), 1e-3, "rel", 8, pad)) == n
    w0 = dq.compress_workspace(p, 0)
    w1 = dq.compress_workspace(p, 1000)
    assert w0 > 0 and w1 - w0 >= 16 * 1000
    assert dq.compress_workspace(p, 10 ** 9) == dq.compress_workspace(p, 20 * 33 * 17)
    assert dq.decompress_workspace(p) >= 4 * (nb + 1)


def test_null_pointers_rejected_before_any_launch(L):
    p = dq.make_params((64,), 1e-3, "abs", 16, "block_mean", 512)
    hp = C.byref(p)
    # x, codes, res, ws missing; pads missing although the mode needs them
    assert L.dq_compress(hp, None, None, None, None, 0, None, None, None, 0, None, None) == dq.DQ_EINVAL
    assert L.dq_decompress(hp, 1e-3, None, None, None, 0, None, None, None, None, 0, None,
                           None) == dq.DQ_EINVAL
    assert L.dq_decompress(hp, -1.0, None, None, None, 0, None, None, None, None, 0, None,
                           None) == dq.DQ_EINVAL
    assert L.dq_result_sync(None, None, None) == dq.DQ_EINVAL


def test_one_hip_runtime_whatever_loads_first():
    """The binding opens libdq.so after torch, so the library binds to torch's
    HIP runtime even when a libdq call comes before any torch use (a second
    runtime in the process could not use torch's streams)."""
    import subprocess
    import sys
    code = ("from paper_2201_04614_amd import binding as dq\n"
            "dq.lib()\n"
            "import torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps').read().splitlines() if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1", r.stdout


def test_noalloc_refuses_oversized_calls_before_any_launch(L):
    """dq_compress_noalloc checks its workspace need against the fixed scratch
    size on the host: an outlier capacity beyond it gives DQ_ENOSCRATCH
    without touching a GPU (none here), the usual checks come first."""
    p = dq.make_params((256, 256, 256), 1e-3, "rel", 8, "zero", 512)
    hp = C.byref(p)
    fake = C.c_void_p(1 << 20)  # never dereferenced: the call returns first
    need = dq.compress_workspace(p, 4 << 20)
    assert need > dq.DQ_SCRATCH_BYTES
    assert L.dq_compress_noalloc(hp, fake, fake, fake, fake, 4 << 20, None, fake, None) == dq.DQ_ENOSCRATCH
    assert L.dq_compress_noalloc(hp, None, fake, fake, fake, 4 << 20, None, fake, None) == dq.DQ_EINVAL
    assert L.dq_compress_noalloc(hp, fake, fake, None, None, 1, None, fake, None) == dq.DQ_EINVAL
    bad = dq.make_params((256, 256, 256), 0.0, "rel", 8, "zero", 512)
    assert L.dq_compress_noalloc(C.byref(bad), fake, fake, fake, fake, 1, None, fake, None) == dq.DQ_EINVAL
    assert dq.compress_workspace(p, 1 << 20) <= dq.DQ_SCRATCH_BYTES


def test_persistent_batch_refusals_on_the_host(L):
    """dq_batch_persistent_workspace plans on the host: a global-mean field
    (its own pass over q) or an outlier capacity below the cell count (dense
    staging only) is DQ_ENOTSUP, a missing output DQ_EINVAL, before any
    device call."""
    from paper_2201_04614_amd import batch as BT
    BT.lib()
    fake = 1 << 24

    def field(shape, pad="zero", cap=None, x_hat=True):
        f = BT.Field()
        f.p = dq.make_params(shape, 1e-3, "rel", 8, pad, 512)
        n = int(np.prod(shape))
        f.x = f.codes = f.out_idx = f.out_val = f.pads = f.cres = f.dres = fake
        f.out_cap = n if cap is None else cap
        f.cws = fake
        f.cws_bytes = dq.compress_workspace(f.p, f.out_cap)
        f.x_hat = fake if x_hat else None
        return f

    need = C.c_uint64(0)
    for fields, want in (([field((64, 64, 64))], dq.DQ_OK),
                         ([field((64, 64, 64)), field((100, 100), pad="global_mean")], dq.DQ_ENOTSUP),
                         ([field((64, 64, 64), cap=1000)], dq.DQ_ENOTSUP),
                         ([field((64, 64, 64), x_hat=False)], dq.DQ_EINVAL)):
        arr = (BT.Field * len(fields))(*fields)
        assert L.dq_batch_persistent_workspace(arr, len(fields), C.byref(need)) == want
    assert need.value > 0
