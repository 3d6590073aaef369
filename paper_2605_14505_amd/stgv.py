"""Python binding of libstgv.so (include/stgv.h): argument marshalling only.

Every function below has the name of the C entry point it calls and does no
arithmetic of the method: all device work runs in the HIP kernels of the
library.  PyTorch provides the device buffers and the HIP stream.  If the
library is not built, importing this module raises.
"""
import ctypes
import math
import os

import torch  # loads the HIP runtime the library then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
# STGV_LIB selects another build of the same library (e.g. one compiled with tuning macros)
LIB_PATH = os.environ.get("STGV_LIB") or os.path.join(_HERE, "lib", "libstgv.so")

LBM_OK, LBM_EINVAL, LBM_ESIZE, LBM_EHIP, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_FORCE_GUO, LBM_FORCE_SHIFT, LBM_FORCE_EDM, LBM_FORCE_HCZ = 0, 1, 2, 3
LBM_FP32, LBM_FP16, LBM_BF16 = 0, 1, 2
LBM_COMPUTE_FP32, LBM_COMPUTE_FP64 = 0, 1
LBM_LAYOUT_AA, LBM_LAYOUT_AB = 0, 1
FORCING = {"guo": LBM_FORCE_GUO, "shift": LBM_FORCE_SHIFT, "edm": LBM_FORCE_EDM, "hcz": LBM_FORCE_HCZ}
STORAGE = {"fp32": LBM_FP32, "fp16": LBM_FP16, "bf16": LBM_BF16}
LAYOUT = {"aa": LBM_LAYOUT_AA, "ab": LBM_LAYOUT_AB}
COMPUTE = {"fp32": LBM_COMPUTE_FP32, "fp64": LBM_COMPUTE_FP64}


class lbm_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("q_f", ctypes.c_int32), ("q_g", ctypes.c_int32),
                ("forcing", ctypes.c_int32), ("storage", ctypes.c_int32), ("compute", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("diag_every", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("u0", ctypes.c_double), ("re", ctypes.c_double), ("fr", ctypes.c_double),
                ("sc", ctypes.c_double), ("g_over_n", ctypes.c_double),
                ("noise_amp", ctypes.c_double), ("seed", ctypes.c_uint64)]


class lbm_diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("ek", ctypes.c_double),
                ("ep", ctypes.c_double), ("eps_k", ctypes.c_double), ("eps_p", ctypes.c_double),
                ("mass", ctypes.c_double), ("scalar", ctypes.c_double),
                ("mom", ctypes.c_double * 3), ("umax", ctypes.c_double),
                ("nonfinite", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "mom"}
        d["mom"] = tuple(self.mom)
        return d


class lbm_post(ctypes.Structure):
    _fields_ = [("gamma_b", ctypes.c_double), ("fr_t", ctypes.c_double), ("r_max", ctypes.c_double),
                ("t_r_max", ctypes.c_double), ("used", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2605_14505_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    sig = {
        "lbm_query_sizes": (ctypes.c_int, [P(lbm_params), P(sz), P(sz)]),
        "lbm_derived": (ctypes.c_int, [P(lbm_params), P(dbl)]),
        "lbm_init_tgv": (ctypes.c_int, [P(lbm_params), vp, sz, vp, sz, vp, P(vp)]),
        "lbm_step": (ctypes.c_int, [vp, i64]),
        "lbm_stream": (ctypes.c_int, [vp, i64]),
        "lbm_sample": (ctypes.c_int, [vp]),
        "lbm_diagnostics": (ctypes.c_int, [vp, P(lbm_diag), i32, P(i32)]),
        "lbm_read_fields": (ctypes.c_int, [vp, vp]),
        "lbm_read_populations": (ctypes.c_int, [vp, vp]),
        "lbm_load_populations": (ctypes.c_int, [vp, vp, i64]),
        "lbm_stencil_info": (ctypes.c_int, [i32, P(i32), P(dbl), P(dbl)]),
        "lbm_bw_probe": (ctypes.c_int, [i32, vp, vp, sz, vp]),
        "lbm_mlp_packed_bytes": (sz, []),
        "lbm_mlp_pack": (ctypes.c_int, [vp, vp, vp, vp]),
        "lbm_mlp_forward": (ctypes.c_int, [vp, vp, i64, vp, vp]),
        "lbm_mlp_grad_work_bytes": (sz, [i64]),
        "lbm_mlp_grad": (ctypes.c_int, [vp, vp, vp, vp, i64, vp, vp, vp, sz, vp]),
        "lbm_mlp_grad_static": (ctypes.c_int, [vp, vp, vp, vp, i64, vp, vp, vp]),
        "lbm_mlp_adam": (ctypes.c_int, [vp, vp, vp, vp, i64, dbl, vp]),
        "lbm_mlp_norm_work_bytes": (sz, []),
        "lbm_mlp_norm": (ctypes.c_int, [vp, vp, i64, vp, vp, sz, vp]),
        "lbm_restrict": (ctypes.c_int, [vp, vp, vp]),
        "lbm_training_pairs": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "lbm_set_mlp": (ctypes.c_int, [vp, vp]),
        "lbm_postprocess": (ctypes.c_int, [P(lbm_diag), i32, dbl, dbl, dbl, P(dbl), P(dbl), P(lbm_post)]),
        "lbm_spectrum_shells": (i32, [i32]),
        "lbm_spectrum_work_bytes": (ctypes.c_int, [i32, P(sz)]),
        "lbm_ke_spectrum": (ctypes.c_int, [vp, vp, sz, vp]),
        "lbm_get_step": (i64, [vp]),
        "lbm_last_error": (ctypes.c_char_p, [vp]),
        "lbm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "lbm_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = res, args
    return lib


LIB = _load()
EXPORTED = ("lbm_query_sizes", "lbm_derived", "lbm_init_tgv", "lbm_step", "lbm_stream", "lbm_sample",
            "lbm_diagnostics", "lbm_read_fields", "lbm_read_populations", "lbm_load_populations",
            "lbm_stencil_info", "lbm_bw_probe", "lbm_get_step", "lbm_last_error",
            "lbm_status_string", "lbm_destroy", "lbm_mlp_packed_bytes", "lbm_mlp_pack",
            "lbm_mlp_forward", "lbm_mlp_grad_work_bytes", "lbm_mlp_grad", "lbm_mlp_grad_static", "lbm_mlp_adam",
            "lbm_mlp_norm_work_bytes", "lbm_mlp_norm", "lbm_restrict", "lbm_training_pairs",
            "lbm_set_mlp", "lbm_postprocess", "lbm_spectrum_shells", "lbm_spectrum_work_bytes",
            "lbm_ke_spectrum")
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS, MLP_NORM = 47, 64, 41, 9897, 135


def _status_name(s):
    return LIB.lbm_status_string(s).decode()


def _check(status, ctx=None):
    if status != LBM_OK:
        raise LbmError(status, LIB.lbm_last_error(ctx).decode())
    return status


def make_params(n, q_f=27, q_g=19, forcing="guo", storage="fp32", compute="fp32", layout="aa",
                diag_every=0, u0=0.05, re=1600.0, fr=1.0, sc=0.7, g_over_n=1.0, noise_amp=0.0,
                seed=0, pad=-1):
    return lbm_params(n=n, q_f=q_f, q_g=q_g, forcing=FORCING.get(forcing, forcing),
                      storage=STORAGE.get(storage, storage), compute=COMPUTE.get(compute, compute),
                      layout=LAYOUT.get(layout, layout), reserved=0,
                      diag_every=diag_every, pad=pad, u0=u0, re=re,
                      fr=math.inf if fr is None else fr, sc=sc, g_over_n=g_over_n,
                      noise_amp=noise_amp, seed=seed)


# --- thin wrappers with the C names ------------------------------------------------
def lbm_query_sizes(p):
    pop, work = ctypes.c_size_t(), ctypes.c_size_t()
    _check(LIB.lbm_query_sizes(ctypes.byref(p), ctypes.byref(pop), ctypes.byref(work)))
    return pop.value, work.value


def lbm_derived(p):
    out = (ctypes.c_double * 8)()
    _check(LIB.lbm_derived(ctypes.byref(p), out))
    return dict(zip(("L", "nu", "D", "tau_f", "tau_g", "nb", "G", "beta"), list(out)))


def lbm_stencil_info(q):
    e = (ctypes.c_int32 * (3 * q))()
    w = (ctypes.c_double * q)()
    cs2 = ctypes.c_double()
    _check(LIB.lbm_stencil_info(q, e, w, ctypes.byref(cs2)))
    return [tuple(e[3 * i:3 * i + 3]) for i in range(q)], list(w), cs2.value


def lbm_init_tgv(p, pop, work, stream):
    ctx = ctypes.c_void_p()
    _check(LIB.lbm_init_tgv(ctypes.byref(p), ctypes.c_void_p(pop.data_ptr()), pop.numel() * pop.element_size(),
                            ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size(),
                            ctypes.c_void_p(stream), ctypes.byref(ctx)))
    return ctx


def lbm_step(ctx, n):
    _check(LIB.lbm_step(ctx, n), ctx)


def lbm_stream(ctx, n):
    _check(LIB.lbm_stream(ctx, n), ctx)


def lbm_sample(ctx):
    _check(LIB.lbm_sample(ctx), ctx)


def lbm_diagnostics(ctx, max_records=4096, raise_unstable=True):
    buf = (lbm_diag * max_records)()
    got = ctypes.c_int32()
    st = LIB.lbm_diagnostics(ctx, buf, max_records, ctypes.byref(got))
    recs = [buf[i].as_dict() for i in range(got.value)]
    if st != LBM_OK and (st != LBM_EUNSTABLE or raise_unstable):
        raise LbmError(st, LIB.lbm_last_error(ctx).decode())
    return recs, st


def lbm_read_fields(ctx, out):
    _check(LIB.lbm_read_fields(ctx, ctypes.c_void_p(out.data_ptr())), ctx)


def lbm_read_populations(ctx, out):
    _check(LIB.lbm_read_populations(ctx, ctypes.c_void_p(out.data_ptr())), ctx)


def lbm_load_populations(ctx, inp, step):
    _check(LIB.lbm_load_populations(ctx, ctypes.c_void_p(inp.data_ptr()), step), ctx)


def lbm_bw_probe(kind, dst, src, nbytes, stream):
    _check(LIB.lbm_bw_probe(kind, ctypes.c_void_p(dst.data_ptr()),
                            ctypes.c_void_p(src.data_ptr() if src is not None else 0),
                            nbytes, ctypes.c_void_p(stream)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def lbm_mlp_packed_bytes():
    return LIB.lbm_mlp_packed_bytes()


def lbm_mlp_pack(params, norm, packed, stream):
    _check(LIB.lbm_mlp_pack(_ptr(params), _ptr(norm), _ptr(packed), ctypes.c_void_p(stream)))


def lbm_mlp_forward(packed, x, rows, y, stream):
    _check(LIB.lbm_mlp_forward(_ptr(packed), _ptr(x), rows, _ptr(y), ctypes.c_void_p(stream)))


def lbm_mlp_grad_work_bytes(batch):
    return LIB.lbm_mlp_grad_work_bytes(batch)


def lbm_mlp_grad(packed, x, y, idx, batch, grad, loss, work, stream):
    _check(LIB.lbm_mlp_grad(_ptr(packed), _ptr(x), _ptr(y), _ptr(idx), batch, _ptr(grad), _ptr(loss),
                            _ptr(work), work.numel() * work.element_size(), ctypes.c_void_p(stream)))


LBM_MLP_STATIC_MAX_BATCH = 16384     # include/stgv.h


def lbm_mlp_grad_static(packed, x, y, idx, batch, grad, loss, stream):
    _check(LIB.lbm_mlp_grad_static(_ptr(packed), _ptr(x), _ptr(y), _ptr(idx), batch, _ptr(grad), _ptr(loss),
                                   ctypes.c_void_p(stream)))


def lbm_mlp_adam(params, m, v, grad, t, lr, stream):
    _check(LIB.lbm_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), t, lr, ctypes.c_void_p(stream)))


def lbm_mlp_norm_work_bytes():
    return LIB.lbm_mlp_norm_work_bytes()


def lbm_mlp_norm(x, y, rows, norm, work, stream):
    _check(LIB.lbm_mlp_norm(_ptr(x), _ptr(y), rows, _ptr(norm), _ptr(work),
                            work.numel() * work.element_size(), ctypes.c_void_p(stream)))


def lbm_restrict(fine_ctx, coarse_ctx, out):
    _check(LIB.lbm_restrict(fine_ctx, coarse_ctx, _ptr(out)), fine_ctx)


def lbm_training_pairs(ctx, a, b, c, x, y):
    _check(LIB.lbm_training_pairs(ctx, _ptr(a), _ptr(b), _ptr(c), _ptr(x), _ptr(y)), ctx)


def lbm_set_mlp(ctx, packed):
    _check(LIB.lbm_set_mlp(ctx, _ptr(packed)), ctx)


def _diag_array(recs):
    arr = (lbm_diag * len(recs))()
    for i, r in enumerate(recs):
        for k, _ in lbm_diag._fields_:
            if k == "mom":
                arr[i].mom[:] = list(r.get("mom", (0.0, 0.0, 0.0)))
            else:
                setattr(arr[i], k, r.get(k, 0))
    return arr


def lbm_postprocess(recs, re, fr, t_end=30.0):
    """recs: diagnostic records (dicts as returned by lbm_diagnostics).  Returns
    (R per record, Gamma per record, bulk summary dict)."""
    n = len(recs)
    arr = _diag_array(recs)
    r_out, g_out, post = (ctypes.c_double * n)(), (ctypes.c_double * n)(), lbm_post()
    _check(LIB.lbm_postprocess(arr, n, re, math.inf if fr is None else fr, t_end, r_out, g_out,
                               ctypes.byref(post)))
    return list(r_out), list(g_out), post.as_dict()


def lbm_spectrum_shells(n):
    return LIB.lbm_spectrum_shells(n)


def lbm_spectrum_work_bytes(n):
    b = ctypes.c_size_t()
    _check(LIB.lbm_spectrum_work_bytes(n, ctypes.byref(b)))
    return b.value


def lbm_ke_spectrum(ctx, work, shells):
    _check(LIB.lbm_ke_spectrum(ctx, _ptr(work), work.numel() * work.element_size(), _ptr(shells)), ctx)


def lbm_get_step(ctx):
    return LIB.lbm_get_step(ctx)


def lbm_destroy(ctx):
    LIB.lbm_destroy(ctx)


# --- buffer ownership helper ----------------------------------------------------------
class Simulation:
    """Owns the torch device buffers of one context; every call goes straight to the C ABI."""

    def __init__(self, device="cuda:0", stream=None, **kw):
        self.params = make_params(**kw)
        self.n = self.params.n
        self.q = self.params.q_f + self.params.q_g
        pop_bytes, work_bytes = lbm_query_sizes(self.params)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # torch's caching allocator returns 512-byte aligned blocks
        self.pop = torch.empty(pop_bytes, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(work_bytes, dtype=torch.uint8, device=self.device)
        self.ctx = lbm_init_tgv(self.params, self.pop, self.work, self.stream.cuda_stream)

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def free_stream(self, n=1):
        """Free streaming (no collision): a measurement and layout check, not the method."""
        lbm_stream(self.ctx, n)

    def sample(self):
        lbm_sample(self.ctx)

    def diagnostics(self, raise_unstable=True):
        return lbm_diagnostics(self.ctx, raise_unstable=raise_unstable)[0]

    def fields(self):
        out = torch.empty((5, self.n, self.n, self.n), dtype=torch.float32, device=self.device)
        lbm_read_fields(self.ctx, out)
        return out

    def populations(self):
        out = torch.empty((self.q, self.n, self.n, self.n), dtype=torch.float32, device=self.device)
        lbm_read_populations(self.ctx, out)
        return out

    def load(self, pops, step=0):
        pops = pops.to(device=self.device, dtype=torch.float32).contiguous()
        assert pops.shape == (self.q, self.n, self.n, self.n)
        lbm_load_populations(self.ctx, pops, step)

    def set_mlp(self, packed):
        """Attach a packed network (a uint8 device tensor kept alive by the caller), or None."""
        self._mlp = packed
        lbm_set_mlp(self.ctx, packed)

    def spectrum(self):
        """Kinetic-energy spectrum E(k), k = 0 .. round(sqrt(3) n / 2), FP64 on the device."""
        if getattr(self, "_spec_work", None) is None:
            self._spec_work = torch.empty(lbm_spectrum_work_bytes(self.n), dtype=torch.uint8, device=self.device)
        out = torch.empty(lbm_spectrum_shells(self.n), dtype=torch.float64, device=self.device)
        lbm_ke_spectrum(self.ctx, self._spec_work, out)
        return out

    def restrict_to(self, coarse):
        """This (fine) state restricted to the grid of `coarse` (a Simulation), FP32 deviations."""
        out = torch.empty((coarse.q, coarse.n, coarse.n, coarse.n), dtype=torch.float32, device=self.device)
        lbm_restrict(self.ctx, coarse.ctx, out)
        return out

    @property
    def step_count(self):
        return lbm_get_step(self.ctx)

    def close(self):
        if self.ctx is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
