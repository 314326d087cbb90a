"""Python binding of libsdint (the C ABI in include/sdint.h).

Argument marshalling only: every function here has the name of the C entry
point it calls, converts Python/NumPy/torch arguments to C types and checks the
status.  All numerical work runs in the HIP library; if ``libsdint.so`` is not
built, every call raises.

PyTorch provides device memory and streams: a context is created on torch's
current stream, and device arguments are torch tensors on that device.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional

import numpy as np

__all__ = [
    "SdiError", "load_library", "library_path", "declared_functions",
    "sdi_ctx_create", "sdi_ctx_destroy", "sdi_last_error", "sdi_device_info",
    "sdi_set_param", "sdi_get_param", "sdi_tune_save", "sdi_tune_load", "sdi_prefactor_feynman", "sdi_lattice_vector",
    "sdi_problem_create", "sdi_problem_from_text", "sdi_problem_from_feynman", "sdi_feynman_sectors", "sdi_text_info", "sdi_problem_destroy", "sdi_problem_norders", "sdi_problem_nsectors", "sdi_problem_sector_origin", "sdi_workspace_bytes",
    "sdi_integrate", "sdi_sector_results", "sdi_evaluate", "sdi_sample_points",
    "sdi_flow_init", "sdi_flow_nparams", "sdi_flow_params", "sdi_flow_set_params", "sdi_flow_sample",
    "sdi_flow_grad", "sdi_flow_set_grad", "sdi_flow_adam", "sdi_flow_train", "sdi_flow_set_active", "sdi_flow_validate",
    "sdi_tune_deformation", "sdi_problem_nvars", "sdi_vegas_refit", "sdi_flow_weights",
    "sdi_sample_points_noalloc", "sdi_checkpoint_export", "sdi_checkpoint_import", "sdi_cubature_regions",
    "sdi_tune_report",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsdint.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "sdint.h")
_lib = None

SDI_CODES = {0: "SDI_OK", -1: "SDI_EINVAL", -2: "SDI_ENOMEM", -3: "SDI_EDEVICE", -4: "SDI_ENOTSUP",
             -5: "SDI_ENONFINITE", -6: "SDI_ESTATE"}
KMAX = 8


class SdiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{SDI_CODES.get(code, code)}: {msg}")
        self.code = code


class SectorDesc(C.Structure):
    _fields_ = [("nvars", C.c_int32), ("nfactors", C.c_int32), ("deform_factor", C.c_int32),
                ("reserved", C.c_int32), ("coeff_re", C.c_double), ("coeff_im", C.c_double),
                ("mono_a", C.POINTER(C.c_double)), ("mono_b", C.POINTER(C.c_double)),
                ("deform_mono", C.POINTER(C.c_int32)), ("fac_nterms", C.POINTER(C.c_int32)),
                ("fac_gamma", C.POINTER(C.c_double)), ("fac_delta", C.POINTER(C.c_double)),
                ("term_coef", C.POINTER(C.c_double)), ("term_exps", C.POINTER(C.c_uint8)),
                ("term_coef_im", C.POINTER(C.c_double))]


class FeynmanDesc(C.Structure):
    _fields_ = [("nvars", C.c_int32), ("loops", C.c_int32), ("d0", C.c_int32), ("order", C.c_int32),
                ("indices", C.POINTER(C.c_int32)), ("u_nterms", C.c_int32), ("f_nterms", C.c_int32),
                ("u_coef", C.POINTER(C.c_double)), ("u_exps", C.POINTER(C.c_uint8)),
                ("f_coef", C.POINTER(C.c_double)), ("f_exps", C.POINTER(C.c_uint8)),
                ("complex_mode", C.c_int32), ("reserved", C.c_int32), ("lam", C.c_double),
                ("f_coef_im", C.POINTER(C.c_double))]


class ProblemDesc(C.Structure):
    _fields_ = [("nsectors", C.c_int32), ("sectors", C.POINTER(SectorDesc)),
                ("order_min", C.c_int32), ("order_max", C.c_int32),
                ("pref_lead", C.c_int32), ("pref_len", C.c_int32),
                ("pref_re", C.POINTER(C.c_double)), ("pref_im", C.POINTER(C.c_double)),
                ("complex_mode", C.c_int32), ("lambda_", C.c_double)]


class Result(C.Structure):
    _fields_ = [("order_min", C.c_int32), ("norders", C.c_int32),
                ("val_re", C.POINTER(C.c_double)), ("val_im", C.POINTER(C.c_double)),
                ("err_re", C.POINTER(C.c_double)), ("err_im", C.POINTER(C.c_double)),
                ("n_evals", C.c_int64), ("n_nonfinite", C.c_int64), ("n_imf_positive", C.c_int64),
                ("ms_sample_eval_reduce", C.c_double), ("ms_refit", C.c_double), ("ms_total", C.c_double),
                ("ms_eval_kernel", C.c_double), ("points_per_thread", C.c_int32), ("blocks", C.c_int32),
                ("tile_log2", C.c_int32), ("waves_per_simd", C.c_int32), ("grouped", C.c_int32),
                ("ms_pilot_kernel", C.c_double), ("pilot_same_kernel", C.c_int32), ("lattice_done", C.c_int64),
                ("cub_regions", C.c_int64), ("cub_rounds", C.c_int32), ("cub_converged", C.c_int32),
                ("ms_flow_train", C.c_double)]


def library_path() -> str:
    return _LIB_PATH


def declared_functions() -> list:
    """Names of the functions include/sdint.h declares."""
    text = open(_HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdi_[a-z_0-9]+)\s*\(", text)))


def load_library():
    """Load libsdint.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build() first")
    try:
        import torch  # noqa: F401  (its HIP runtime is the one the library binds to)
    except ImportError:
        pass
    lib = C.CDLL(_LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "sdi_ctx_create": (C.c_int, [C.c_int, vp, C.POINTER(vp)]),
        "sdi_ctx_destroy": (None, [vp]),
        "sdi_last_error": (C.c_char_p, [vp]),
        "sdi_device_info": (C.c_int, [vp, C.c_char_p, C.c_size_t]),
        "sdi_set_param": (C.c_int, [vp, C.c_char_p, C.c_char_p]),
        "sdi_get_param": (C.c_int, [vp, C.c_char_p, C.c_char_p, C.c_size_t]),
        "sdi_tune_save": (C.c_int, [vp, C.c_char_p]),
        "sdi_tune_load": (C.c_int, [vp, C.c_char_p]),
        "sdi_prefactor_feynman": (C.c_int, [i32, C.POINTER(i32), i32, i32, i32, C.POINTER(i32), dp]),
        "sdi_lattice_vector": (C.c_int, [i32, i32, C.POINTER(C.c_uint32)]),
        "sdi_problem_create": (C.c_int, [vp, C.POINTER(ProblemDesc), C.POINTER(vp)]),
        "sdi_problem_from_text": (C.c_int, [vp, C.c_char_p, C.POINTER(vp)]),
        "sdi_problem_from_feynman": (C.c_int, [vp, C.POINTER(FeynmanDesc), C.POINTER(vp)]),
        "sdi_feynman_sectors": (C.c_int, [C.POINTER(FeynmanDesc), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32)]),
        "sdi_text_info": (C.c_int, [C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                    C.c_char_p, C.c_size_t]),
        "sdi_problem_destroy": (None, [vp]),
        "sdi_problem_norders": (C.c_int, [vp]),
        "sdi_problem_nsectors": (C.c_int, [vp]),
        "sdi_problem_sector_origin": (C.c_int, [vp, i32]),
        "sdi_problem_nvars": (C.c_int, [vp, i32]),
        "sdi_sample_points_noalloc": (C.c_int, [vp, vp, i32, i32, i64, i64, vp, vp]),
        "sdi_checkpoint_export": (C.c_int, [vp, vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]),
        "sdi_checkpoint_import": (C.c_int, [vp, vp, vp, C.c_size_t]),
        "sdi_tune_report": (C.c_int, [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
        "sdi_cubature_regions": (C.c_int, [vp, vp, i64, C.POINTER(C.c_int64), vp, vp, vp, vp, vp, vp]),
        "sdi_vegas_refit": (C.c_int, [vp, i32, i32, i32, vp, vp, C.c_double]),
        "sdi_flow_weights": (C.c_int, [vp, i64, i32, vp, vp, dp, vp]),
        "sdi_workspace_bytes": (C.c_size_t, [vp, vp]),
        "sdi_integrate": (C.c_int, [vp, vp, vp, C.c_size_t, C.POINTER(Result)]),
        "sdi_sector_results": (C.c_int, [vp, vp, i32, dp, dp, dp, C.POINTER(i64)]),
        "sdi_evaluate": (C.c_int, [vp, vp, i32, vp, i64, vp, vp]),
        "sdi_sample_points": (C.c_int, [vp, vp, i32, i32, i64, i64, vp, vp]),
        "sdi_tune_deformation": (C.c_int, [vp, vp, C.c_double, i32, i32, i32, dp]),
        "sdi_flow_init": (C.c_int, [vp, vp, C.c_uint64]),
        "sdi_flow_nparams": (i64, [vp, i32]),
        "sdi_flow_params": (C.c_int, [vp, vp, i32, C.POINTER(C.c_float), i64]),
        "sdi_flow_set_params": (C.c_int, [vp, vp, i32, C.POINTER(C.c_float), i64]),
        "sdi_flow_sample": (C.c_int, [vp, vp, i32, vp, i64, vp, vp]),
        "sdi_flow_grad": (C.c_int, [vp, vp, i32, vp, vp, i64, C.POINTER(C.c_float)]),
        "sdi_flow_set_grad": (C.c_int, [vp, vp, i32, C.POINTER(C.c_float), i64]),
        "sdi_flow_adam": (C.c_int, [vp, vp, C.c_double]),
        "sdi_flow_train": (C.c_int, [vp, vp, C.POINTER(i32), i32, i32, i32, C.c_double, C.POINTER(C.c_double),
                                     C.POINTER(C.c_float)]),
        "sdi_flow_set_active": (C.c_int, [vp, vp, i32, i32]),
        "sdi_flow_validate": (C.c_int, [vp, vp, i32, C.POINTER(C.c_double), C.POINTER(i32), C.POINTER(C.c_float)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, ctx=None, allow=()):
    if rc != 0 and rc not in allow:
        msg = load_library().sdi_last_error(ctx).decode() if ctx else ""
        raise SdiError(rc, msg)
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------- context

def sdi_ctx_create(device: int = 0, stream: Optional[int] = None):
    """Context on `device`; stream defaults to torch's current stream on it."""
    lib = load_library()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(device).cuda_stream
    h = C.c_void_p()
    _check(lib.sdi_ctx_create(device, C.c_void_p(stream), C.byref(h)))
    _CTX_DEVICE[h.value] = device
    return h


_CTX_DEVICE = {}   # context -> device ordinal, for checking device arguments


def _device_tensor(ctx, t, name: str, shape):
    """Checks a device argument before its pointer goes to the library (which
    cannot check the size of a buffer): fp64, on the context's device,
    contiguous, of the given shape (None = any extent)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise SdiError(-1, f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise SdiError(-1, f"{name} must be float64, got {t.dtype}")
    dev = _CTX_DEVICE.get(ctx.value if hasattr(ctx, "value") else ctx)
    if not t.is_cuda or (dev is not None and t.device.index != dev):
        raise SdiError(-1, f"{name} must be on cuda:{dev}, got {t.device}")
    if t.dim() != len(shape) or any(w is not None and t.shape[i] != w for i, w in enumerate(shape)):
        raise SdiError(-1, f"{name} must have shape {tuple('*' if w is None else w for w in shape)}, "
                           f"got {tuple(t.shape)}")
    return t.contiguous()


def sdi_problem_nvars(prob, s: int) -> int:
    return _check_count(load_library().sdi_problem_nvars(prob, s))


def sdi_ctx_destroy(ctx):
    load_library().sdi_ctx_destroy(ctx)


def sdi_last_error(ctx) -> str:
    return load_library().sdi_last_error(ctx).decode()


def sdi_device_info(ctx) -> str:
    buf = C.create_string_buffer(512)
    _check(load_library().sdi_device_info(ctx, buf, 512), ctx)
    return buf.value.decode()


def sdi_set_param(ctx, key: str, value):
    _check(load_library().sdi_set_param(ctx, key.encode(), str(value).encode()), ctx)


def sdi_get_param(ctx, key: str) -> str:
    buf = C.create_string_buffer(64)
    _check(load_library().sdi_get_param(ctx, key.encode(), buf, 64), ctx)
    return buf.value.decode()


def sdi_tune_report(ctx) -> str:
    """Candidates and times of the last autotuner search (text, one line each)."""
    lib = load_library()
    need = C.c_size_t(0)
    _check(lib.sdi_tune_report(ctx, None, 0, C.byref(need)), ctx)
    buf = C.create_string_buffer(need.value)
    _check(lib.sdi_tune_report(ctx, buf, need.value, C.byref(need)), ctx)
    return buf.value.decode()


def sdi_tune_save(ctx, path: str):
    _check(load_library().sdi_tune_save(ctx, os.fsencode(path)), ctx)


def sdi_tune_load(ctx, path: str) -> int:
    """Number of autotuner decisions loaded (0 for a file of another kernel build)."""
    rc = load_library().sdi_tune_load(ctx, os.fsencode(path))
    if rc < 0:
        _check(rc, ctx)
    return int(rc)


def sdi_prefactor_feynman(loops: int, indices, d0: int, length: int):
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    out = np.zeros(length)
    lead = C.c_int32()
    _check(load_library().sdi_prefactor_feynman(loops, idx.ctypes.data_as(C.POINTER(C.c_int32)), len(idx), d0,
                                                length, C.byref(lead), _dptr(out)))
    return int(lead.value), out


def sdi_lattice_vector(m: int, dims: int) -> np.ndarray:
    out = np.zeros(dims, dtype=np.uint32)
    _check(load_library().sdi_lattice_vector(m, dims, out.ctypes.data_as(C.POINTER(C.c_uint32))))
    return out


# ---------------------------------------------------------------- problem

def _prefactor_of(problem):
    """Prefactor series of a sectorgen.Problem (explicit, or expanded by the library)."""
    if problem.feynman is None:
        p = np.asarray(problem.pref, dtype=np.complex128)
        return problem.pref_lead, p.real.copy(), p.imag.copy()
    f = problem.feynman
    lead, _ = sdi_prefactor_feynman(f.loops, f.indices, f.d0, 1)
    # singular variables after the library's reduction of a_j < -1 (integer a_j <= -1 end at -1)
    max_s = max(int(np.sum((s.a <= -1.0) & (s.a == np.floor(s.a)))) for s in problem.sectors)
    length = max(1, problem.order_max - lead + max_s + 1)
    lead, ser = sdi_prefactor_feynman(f.loops, f.indices, f.d0, length)
    return lead, ser, np.zeros_like(ser)


def sdi_problem_create(ctx, problem):
    """Compile a sectorgen.Problem into the library (copies every input)."""
    keep = []
    descs = (SectorDesc * len(problem.sectors))()
    for i, s in enumerate(problem.sectors):
        a = np.ascontiguousarray(s.a, dtype=np.float64)
        b = np.ascontiguousarray(s.b, dtype=np.float64)
        nt = np.array([len(f.coef) for f in s.factors], dtype=np.int32)
        g = np.array([f.gamma for f in s.factors], dtype=np.float64)
        d = np.array([f.delta for f in s.factors], dtype=np.float64)
        allc = np.concatenate([np.asarray(f.coef) for f in s.factors]) if s.factors else np.zeros(0)
        coef = np.ascontiguousarray(allc.real, dtype=np.float64)
        # imaginary parts of the term coefficients (complex mode), passed only when some is nonzero
        coef_im = (np.ascontiguousarray(allc.imag, dtype=np.float64)
                   if np.iscomplexobj(allc) and np.any(allc.imag != 0) else None)
        exps = np.ascontiguousarray(np.concatenate([f.exps for f in s.factors]).astype(np.uint8)
                                    if s.factors else np.zeros((0, s.n), np.uint8))
        dm = (np.ascontiguousarray(s.deform_mono, dtype=np.int32) if s.deform_mono is not None else None)
        keep += [a, b, nt, g, d, coef, exps, dm, coef_im]
        c = complex(s.coeff)
        descs[i] = SectorDesc(
            s.n, len(s.factors), s.deform_factor, 0, c.real, c.imag, _dptr(a), _dptr(b),
            dm.ctypes.data_as(C.POINTER(C.c_int32)) if dm is not None else None,
            nt.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(g), _dptr(d), _dptr(coef),
            exps.ctypes.data_as(C.POINTER(C.c_uint8)), _dptr(coef_im) if coef_im is not None else None)
    lead, pre, pim = _prefactor_of(problem)
    pre = np.ascontiguousarray(pre, dtype=np.float64)
    pim = np.ascontiguousarray(pim, dtype=np.float64)
    keep += [pre, pim]
    pd = ProblemDesc(len(problem.sectors), descs, problem.order_min, problem.order_max, lead, len(pre),
                     _dptr(pre), _dptr(pim), int(problem.complex_mode), float(problem.lam))
    h = C.c_void_p()
    _check(load_library().sdi_problem_create(ctx, C.byref(pd), C.byref(h)), ctx)
    return h


def _feynman_desc(U: dict, F: dict, loops: int, indices, order: int, d0: int, complex_mode: bool, lam: float):
    """Descriptor of SDEvaluate[{U, F, l}, indices, order]; U and F as {exponent tuple: coefficient}."""
    n = len(indices)
    keep = []

    def arrays(p):
        vals = [complex(c) for c in p.values()]
        coef = np.ascontiguousarray([c.real for c in vals], dtype=np.float64)
        im = np.ascontiguousarray([c.imag for c in vals], dtype=np.float64)
        exps = np.ascontiguousarray(np.array(list(p.keys()), dtype=np.uint8).reshape(len(p), n))
        keep.extend([coef, im, exps])
        return len(p), _dptr(coef), exps.ctypes.data_as(C.POINTER(C.c_uint8)), (_dptr(im) if im.any() else None)

    idx = np.ascontiguousarray(indices, dtype=np.int32)
    keep.append(idx)
    un, uc, ue, ui = arrays(U)
    if ui is not None:
        raise SdiError(-1, "U has real coefficients")
    fn, fc, fe, fi = arrays(F)
    d = FeynmanDesc(n, loops, d0, order, idx.ctypes.data_as(C.POINTER(C.c_int32)), un, fn, uc, ue, fc, fe,
                    int(complex_mode), 0, float(lam), fi)
    return d, keep


def sdi_problem_from_feynman(ctx, U: dict, F: dict, loops: int, indices, order: int, d0: int = 4,
                             complex_mode: bool = False, lam: float = 0.0):
    """Compile a Feynman integral from its Symanzik polynomials (the library decomposes it)."""
    d, keep = _feynman_desc(U, F, loops, indices, order, d0, complex_mode, lam)
    h = C.c_void_p()
    _check(load_library().sdi_problem_from_feynman(ctx, C.byref(d), C.byref(h)), ctx)
    del keep
    return h


def sdi_feynman_sectors(U: dict, F: dict, loops: int, indices, d0: int = 4):
    """(sectors, lowest result order, variables per sector) of the decomposition, host only."""
    cplx = any(complex(c).imag != 0.0 for c in F.values())      # complex masses: a complex-mode input
    d, keep = _feynman_desc(U, F, loops, indices, 0, d0, cplx, 0.0)
    ns, om, nv = C.c_int32(), C.c_int32(), C.c_int32()
    rc = load_library().sdi_feynman_sectors(C.byref(d), C.byref(ns), C.byref(om), C.byref(nv))
    if rc != 0:
        raise SdiError(rc, "feynman decomposition failed")
    del keep
    return ns.value, om.value, nv.value


def sdi_problem_from_text(ctx, text: str):
    """Compile an integrand in the workers' text format (one sector, one order)."""
    h = C.c_void_p()
    _check(load_library().sdi_problem_from_text(ctx, text.encode(), C.byref(h)), ctx)
    return h


def sdi_text_info(text: str) -> dict:
    """Host-only compile of a text integrand: {"nvars", "ninstructions", "nslots"};
    raises SdiError with the parser's message on failure."""
    n, ni, ns = C.c_int32(), C.c_int64(), C.c_int32()
    buf = C.create_string_buffer(512)
    rc = load_library().sdi_text_info(text.encode(), C.byref(n), C.byref(ni), C.byref(ns), buf, 512)
    if rc != 0:
        raise SdiError(rc, buf.value.decode())
    return {"nvars": n.value, "ninstructions": ni.value, "nslots": ns.value}


def sdi_problem_destroy(prob):
    load_library().sdi_problem_destroy(prob)


def sdi_problem_nsectors(prob) -> int:
    return _check_count(load_library().sdi_problem_nsectors(prob))


def _check_count(v: int) -> int:
    if v < 0:
        raise SdiError(v, "invalid problem handle")
    return int(v)


def sdi_problem_norders(prob) -> int:
    return int(load_library().sdi_problem_norders(prob))


def sdi_problem_sector_origin(prob, s: int) -> int:
    """Input sector of compiled sector s (sectors with a_j < -1 are expanded)."""
    return _check_count(int(load_library().sdi_problem_sector_origin(prob, s)))


def sdi_workspace_bytes(ctx, prob) -> int:
    return int(load_library().sdi_workspace_bytes(ctx, prob))


# ---------------------------------------------------------------- integrate

def sdi_integrate(ctx, prob, workspace=None) -> dict:
    """Run the integrator; `workspace` is an optional torch uint8 cuda tensor."""
    K = sdi_problem_norders(prob)
    arrs = [np.zeros(K) for _ in range(4)]
    res = Result(0, K, *[_dptr(x) for x in arrs], 0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0, 0, 0.0, 0, 0, 0, 0, 0, 0.0)
    ptr, nbytes = (None, 0) if workspace is None else (C.c_void_p(workspace.data_ptr()), workspace.numel())
    if workspace is not None:
        import torch
        torch.cuda.current_stream(workspace.device).synchronize()
    rc = _check(load_library().sdi_integrate(ctx, prob, ptr, nbytes, C.byref(res)), ctx, allow=(-5,))
    return {"status": rc, "order_min": res.order_min, "value": arrs[0] + 1j * arrs[1],
            "err_re": arrs[2], "err_im": arrs[3], "n_evals": res.n_evals, "n_nonfinite": res.n_nonfinite,
            "n_imf_positive": res.n_imf_positive, "ms_final": res.ms_sample_eval_reduce,
            "ms_warmup": res.ms_refit, "ms_total": res.ms_total, "ms_eval_kernel": res.ms_eval_kernel,
            "ppt": res.points_per_thread, "blocks": res.blocks, "tile_log2": res.tile_log2,
            "waves_per_simd": res.waves_per_simd, "grouped": res.grouped, "ms_pilot_kernel": res.ms_pilot_kernel,
            "pilot_same_kernel": res.pilot_same_kernel, "lattice_done": res.lattice_done,
            "cub_regions": res.cub_regions, "cub_rounds": res.cub_rounds, "cub_converged": res.cub_converged,
            "ms_flow_train": res.ms_flow_train}


def sdi_sector_results(ctx, prob, s: int, nshifts: int):
    K = sdi_problem_norders(prob)
    mean = np.zeros((K, 2))
    err = np.zeros((K, 2))
    per = np.zeros((nshifts, K, 2))
    nev = C.c_int64()
    _check(load_library().sdi_sector_results(ctx, prob, s, _dptr(mean), _dptr(err), _dptr(per), C.byref(nev)), ctx)
    return mean[:, 0] + 1j * mean[:, 1], err, per[..., 0] + 1j * per[..., 1], int(nev.value)


def sdi_evaluate(ctx, prob, s: int, x, with_cond: bool = False):
    """x: torch float64 cuda tensor (npts, n); returns a cuda tensor (npts, K, 2),
    and with_cond also the per-order sums of |term| (npts, K)."""
    import torch
    K = sdi_problem_norders(prob)
    x = _device_tensor(ctx, x, "x", (None, sdi_problem_nvars(prob, s)))
    out = torch.empty((x.shape[0], K, 2), dtype=torch.float64, device=x.device)
    cond = torch.empty((x.shape[0], K), dtype=torch.float64, device=x.device) if with_cond else None
    torch.cuda.current_stream(x.device).synchronize()
    _check(load_library().sdi_evaluate(ctx, prob, s, C.c_void_p(x.data_ptr()), x.shape[0],
                                       C.c_void_p(out.data_ptr()),
                                       C.c_void_p(cond.data_ptr()) if with_cond else None), ctx)
    return (out, cond) if with_cond else out


def sdi_sample_points(ctx, prob, s: int, shift: int, i0: int, npts: int, nvars: int, device=0):
    import torch
    x = torch.empty((npts, nvars), dtype=torch.float64, device=f"cuda:{device}")
    w = torch.empty((npts,), dtype=torch.float64, device=f"cuda:{device}")
    torch.cuda.current_stream(device).synchronize()
    _check(load_library().sdi_sample_points(ctx, prob, s, shift, i0, npts, C.c_void_p(x.data_ptr()),
                                            C.c_void_p(w.data_ptr())), ctx)
    return x, w


def sdi_vegas_refit(ctx, hist, grid, alpha: float = 1.5):
    """One Vegas refit on the device: hist (n, nbins, k) float64 cuda tensor of
    per-bin sums of |w f_k|^2, grid (n, nbins + 1) edges, refitted in place."""
    import torch
    n, nb, k = hist.shape
    hist = _device_tensor(ctx, hist, "hist", (n, nb, k))
    if not grid.is_contiguous():
        raise SdiError(-1, "grid must be contiguous (it is updated in place)")
    _device_tensor(ctx, grid, "grid", (n, nb + 1))
    torch.cuda.current_stream(grid.device).synchronize()
    _check(load_library().sdi_vegas_refit(ctx, n, nb, k, C.c_void_p(hist.data_ptr()), C.c_void_p(grid.data_ptr()),
                                          float(alpha)), ctx)
    return grid


def sdi_flow_weights(ctx, f, lq, order_weights=None):
    """Training loss weights on the device: f (npts, K, 2) and lq (npts,) float64 cuda tensors."""
    import torch
    npts, K = f.shape[0], f.shape[1]
    f = _device_tensor(ctx, f, "f", (npts, K, 2))
    lq = _device_tensor(ctx, lq, "lq", (npts,))
    c = torch.empty((npts,), dtype=torch.float64, device=f.device)
    w = None if order_weights is None else np.ascontiguousarray(order_weights, dtype=np.float64)
    if w is not None and w.shape != (K,):
        raise ValueError("order_weights needs one weight per order")
    torch.cuda.current_stream(f.device).synchronize()
    _check(load_library().sdi_flow_weights(ctx, npts, K, C.c_void_p(f.data_ptr()), C.c_void_p(lq.data_ptr()),
                                           _dptr(w) if w is not None else None, C.c_void_p(c.data_ptr())), ctx)
    return c


def sdi_sample_points_noalloc(ctx, prob, s: int, shift: int, i0: int, x, w=None):
    """sdi_sample_points into caller tensors x (npts, n) and w (npts,) (float64 on the
    context's device), through the entry point that allocates no device memory."""
    import torch
    n = sdi_problem_nvars(prob, s)
    x = _device_tensor(ctx, x, "x", (None, n))
    if w is not None:
        w = _device_tensor(ctx, w, "w", (x.shape[0],))
    torch.cuda.current_stream(x.device).synchronize()
    _check(load_library().sdi_sample_points_noalloc(ctx, prob, s, shift, i0, x.shape[0], C.c_void_p(x.data_ptr()),
                                                    C.c_void_p(w.data_ptr()) if w is not None else None), ctx)
    return x, w


def sdi_cubature_regions(ctx, prob) -> dict:
    """Regions of the last cubature run (sector, level, index, value, error, axis)."""
    lib = load_library()
    n = C.c_int64(0)
    _check(lib.sdi_cubature_regions(ctx, prob, 0, C.byref(n), None, None, None, None, None, None), ctx)
    K = sdi_problem_norders(prob)
    N = n.value
    sec = np.zeros(N, np.int32)
    lev = np.zeros((N, 16), np.uint8)
    idx = np.zeros((N, 16), np.uint32)
    val = np.zeros((N, K, 2))
    err = np.zeros((N, K, 2))
    axis = np.zeros(N, np.int32)
    _check(lib.sdi_cubature_regions(ctx, prob, N, C.byref(n), sec.ctypes.data, lev.ctypes.data, idx.ctypes.data,
                                    val.ctypes.data, err.ctypes.data, axis.ctypes.data), ctx)
    return {"sector": sec, "level": lev, "index": idx, "value": val[..., 0] + 1j * val[..., 1],
            "err_re": err[..., 0], "err_im": err[..., 1], "axis": axis}


def sdi_checkpoint_export(ctx, prob) -> bytes:
    """The resumable pass's sums and progress as bytes."""
    lib = load_library()
    need = C.c_size_t(0)
    _check(lib.sdi_checkpoint_export(ctx, prob, None, 0, C.byref(need)), ctx)
    buf = C.create_string_buffer(need.value)
    _check(lib.sdi_checkpoint_export(ctx, prob, buf, need.value, C.byref(need)), ctx)
    return buf.raw[: need.value]


def sdi_checkpoint_import(ctx, prob, data: bytes):
    buf = C.create_string_buffer(bytes(data), len(data))
    _check(load_library().sdi_checkpoint_import(ctx, prob, buf, len(data)), ctx)


# ---------------------------------------------------------------- deformation size

def sdi_tune_deformation(ctx, prob, lambda_max: float, split: int = 4, points_log2: int = 10,
                         conservative: bool = False) -> np.ndarray:
    """Chooses every sector's deformation size on the GPU; returns them (host array)."""
    out = np.zeros(sdi_problem_nsectors(prob), dtype=np.float64)
    _check(load_library().sdi_tune_deformation(ctx, prob, float(lambda_max), split, points_log2,
                                               1 if conservative else 0, _dptr(out)), ctx)
    return out


# ---------------------------------------------------------------- learned sampler

def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def sdi_flow_init(ctx, prob, seed: int):
    _check(load_library().sdi_flow_init(ctx, prob, seed & 0xFFFFFFFFFFFFFFFF), ctx)


def sdi_flow_nparams(prob, s: int) -> int:
    n = load_library().sdi_flow_nparams(prob, s)
    if n < 0:
        raise SdiError(int(n), "no flow or sector out of range")
    return int(n)


def sdi_flow_params(ctx, prob, s: int) -> np.ndarray:
    out = np.empty(sdi_flow_nparams(prob, s), dtype=np.float32)
    _check(load_library().sdi_flow_params(ctx, prob, s, _fptr(out), out.size), ctx)
    return out


def sdi_flow_set_params(ctx, prob, s: int, values):
    v = np.ascontiguousarray(values, dtype=np.float32)
    _check(load_library().sdi_flow_set_params(ctx, prob, s, _fptr(v), v.size), ctx)


def sdi_flow_sample(ctx, prob, s: int, u):
    """u: torch float64 cuda tensor (npts, n); returns (x, log q) cuda tensors."""
    import torch
    u = _device_tensor(ctx, u, "u", (None, sdi_problem_nvars(prob, s)))
    x = torch.empty_like(u)
    lq = torch.empty((u.shape[0],), dtype=torch.float64, device=u.device)
    torch.cuda.current_stream(u.device).synchronize()
    _check(load_library().sdi_flow_sample(ctx, prob, s, C.c_void_p(u.data_ptr()), u.shape[0],
                                          C.c_void_p(x.data_ptr()), C.c_void_p(lq.data_ptr())), ctx)
    return x, lq


def sdi_flow_grad(ctx, prob, s: int, x, c) -> np.ndarray:
    """x: (npts, n), c: (npts,) torch float64 cuda tensors; returns the fp32 gradient."""
    import torch
    x = _device_tensor(ctx, x, "x", (None, sdi_problem_nvars(prob, s)))
    c = _device_tensor(ctx, c, "c", (x.shape[0],))
    g = np.empty(sdi_flow_nparams(prob, s), dtype=np.float32)
    torch.cuda.current_stream(x.device).synchronize()
    _check(load_library().sdi_flow_grad(ctx, prob, s, C.c_void_p(x.data_ptr()), C.c_void_p(c.data_ptr()),
                                        x.shape[0], _fptr(g)), ctx)
    return g


def sdi_flow_set_grad(ctx, prob, s: int, values):
    v = np.ascontiguousarray(values, dtype=np.float32)
    _check(load_library().sdi_flow_set_grad(ctx, prob, s, _fptr(v), v.size), ctx)


def sdi_flow_adam(ctx, prob, lr: float):
    _check(load_library().sdi_flow_adam(ctx, prob, float(lr)), ctx)


def _order_weights(prob, order_weights):
    if order_weights is None:
        return None, None
    w = np.ascontiguousarray(order_weights, dtype=np.float64)
    if w.shape != (sdi_problem_norders(prob),):
        raise ValueError("order_weights needs one weight per result order")
    return w, _dptr(w)


def sdi_flow_train(ctx, prob, iters: int, batch_log2: int, lr: float, sectors=None, order_weights=None) -> float:
    """Trains the flows of `sectors` (all if None) on the GPU; returns the device time in ms."""
    ms = C.c_float(0.0)
    if sectors is None:
        ptr, n = None, 0
    else:
        sel = np.ascontiguousarray(sectors, dtype=np.int32)
        ptr, n = sel.ctypes.data_as(C.POINTER(C.c_int32)), sel.size
    w, wp = _order_weights(prob, order_weights)
    _check(load_library().sdi_flow_train(ctx, prob, ptr, n, iters, batch_log2, float(lr), wp, C.byref(ms)), ctx)
    return float(ms.value)


def sdi_flow_set_active(ctx, prob, s: int, active: bool):
    _check(load_library().sdi_flow_set_active(ctx, prob, s, 1 if active else 0), ctx)


def sdi_flow_validate(ctx, prob, lattice_log2: int, order_weights=None):
    """Deactivates flows that do not lower their sector's share of the relative errors; returns (kept, device ms)."""
    kept = np.zeros(sdi_problem_nsectors(prob), dtype=np.int32)
    ms = C.c_float(0.0)
    w, wp = _order_weights(prob, order_weights)
    _check(load_library().sdi_flow_validate(ctx, prob, lattice_log2, wp, kept.ctypes.data_as(C.POINTER(C.c_int32)),
                                            C.byref(ms)), ctx)
    return kept.astype(bool), float(ms.value)
