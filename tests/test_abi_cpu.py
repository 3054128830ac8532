"""CPU-side checks of the C ABI: the HIP library loads and exports every entry point
include/nlse.h declares, and the binding's struct matches the header's layout.
No GPU work is launched here."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(nlse_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    import paper_1109_1027_amd as P
    lib = P.load()
    names = declared()
    assert {"nlse_create", "nlse_set_field", "nlse_step", "nlse_get_field", "nlse_mass"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_params_struct_layout():
    """nlse_params: int32 ndim; int64 n[3]; double h, a, s; const double *V; int32 bc, prec,
    allow_unstable; void *stream  ->  offsets as a C compiler lays them out."""
    from paper_1109_1027_amd.nlse import Params
    assert Params.n.offset == 8
    assert Params.h.offset == 32
    assert Params.V.offset == 56
    assert Params.bc.offset == 64
    assert Params.stream.offset == 80
    assert ctypes.sizeof(Params) == 88


def test_no_gpu_gives_error_not_crash():
    """Without a GPU the library reports an error code instead of faulting (and never falls back)."""
    import torch
    if torch.cuda.is_available():
        return
    import paper_1109_1027_amd as P
    try:
        P.Solver(2, 8, 0.1, 1.0, 1.0, stream=None)
    except P.NLSEError as e:
        assert e.code in (-4, -5)
    else:
        raise AssertionError("expected an error without a GPU")


def test_committed_corrector_weights_load():
    import numpy as np
    from paper_1109_1027_amd import corrector as K
    p, scale = K.load_weights()
    assert p.dtype == np.float32 and p.size == 32 * 9 * 8 + 32 + 32 * 9 * 32 + 32 + 2 * 9 * 32 + 2
    assert np.all(np.isfinite(p)) and 0 < scale < 1


def test_parameter_validation_before_any_allocation():
    """nlse_create and nlse_batch_create reject invalid problems with their documented codes before
    touching the device, so this runs without a GPU."""
    import numpy as np
    import nlse_inputs as I
    import paper_1109_1027_amd as P
    bad = [dict(ndim=4, n=8, h=0.1, a=1.0, s=1.0),            # ndim
           dict(ndim=2, n=1, h=0.1, a=1.0, s=1.0),            # fewer than 2 intervals
           dict(ndim=2, n=8, h=0.0, a=1.0, s=1.0),            # h
           dict(ndim=2, n=8, h=0.1, a=-1.0, s=1.0),           # a > 0 required
           dict(ndim=2, n=8, h=0.1, a=1.0, s=float("nan")),   # s finite
           dict(ndim=1, n=3, h=0.1, a=1.0, s=1.0, bc="msd")]  # 1D MSD needs n >= 4
    for kw in bad:
        try:
            P.Solver(kw.pop("ndim"), kw.pop("n"), kw.pop("h"), kw.pop("a"), kw.pop("s"), stream=None, **kw)
        except P.NLSEError as e:
            assert e.code == -1, (e.code, e)
        else:
            raise AssertionError("invalid parameters accepted")
    for prec, n in (("f64", 5120), ("f32", 9216), ("mixed", 9216)):   # one node beyond the 1D on-chip limit
        try:
            P.Solver(1, n, 0.01, 1.0, 1.0, stream=None, prec=prec)
        except P.NLSEError as e:
            assert e.code == -6, (prec, n, e.code, e)
        else:
            raise AssertionError("1D field beyond the on-chip solver accepted")
    for args, code in (((3, 1300, 0.1, 1.0, 1.0), -6),             # 3D beyond 32-bit offsets
                       ((3, (2000, 1000, 1200), 0.1, 1.0, 1.0), -6),
                       ((2, 10 ** 9, 0.1, 1.0, 1.0), -4)):          # no device holds it
        try:
            P.Solver(*args, stream=None)
        except P.NLSEError as e:
            assert e.code == code, (args, e.code, e)
        else:
            raise AssertionError("oversized field accepted")
    g3 = I.grid(3, 8, -1.0, 1.0)
    g2 = I.grid(2, 8, -1.0, 1.0)
    for spec, code in ((I.ProblemSpec("a", g3, 0.5, -1.0, None, np.zeros(g3.shape, complex)), -6),
                       (I.ProblemSpec("b", g2, 0.5, -1.0, None, np.zeros(g2.shape, complex), "msd"), -6)):
        try:
            P.Batch([spec], prec="f32", stream=None)
        except P.NLSEError as e:
            assert e.code == code, (e.code, e)
        else:
            raise AssertionError("unsupported batch accepted")
