"""Python binding of libdkss (DKSS multiplication on one MI355X).

Argument marshalling only: every step of the multiplication runs in the HIP kernels of
``csrc/libdkss.so``; this module passes device pointers, lengths, parameter structs and the
current HIP stream through the C ABI declared in ``include/dkss.h``.  PyTorch provides device
memory and streams.  Integers are torch.int32 CUDA tensors holding uint32 limbs, least
significant limb first.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "csrc", "libdkss.so")

POLICY_THESIS = 0
POLICY_TUNED = 1
POLICY_LEARNED = 2

OK, EINVAL, ENOSPC, ERANGE, EHIP, ENOTIMPL, ETOOBIG = 0, -1, -2, -3, -4, -5, -6
NOALLOC_SCRATCH_BYTES = 128 << 20


class DkssError(RuntimeError):
    def __init__(self, code, what):
        msg = "%s: %s (%d)" % (what, lib().dkss_strerror(code).decode(), code)
        if code == EHIP:
            h = lib().dkss_last_hip_error()
            msg += "; HIP error %d: %s" % (h, lib().dkss_hip_error_string(h).decode())
        super().__init__(msg)
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("log2_M", ctypes.c_uint32), ("log2_m", ctypes.c_uint32), ("u", ctypes.c_uint32),
                ("p_bits", ctypes.c_uint32), ("z", ctypes.c_uint32),
                ("n_levels", ctypes.c_uint32), ("radix_log2", ctypes.c_uint32 * 8),
                ("cutoff_bits", ctypes.c_uint64)]

    @classmethod
    def make(cls, log2_M, log2_m, u=0, p_bits=128, z=1, radices=None, cutoff_bits=0):
        p = cls()
        p.log2_M, p.log2_m, p.u, p.p_bits, p.z = log2_M, log2_m, u, p_bits, z
        radices = list(radices or [])
        p.n_levels = len(radices)
        for i, r in enumerate(radices):
            p.radix_log2[i] = r
        p.cutoff_bits = cutoff_bits
        return p

    def as_dict(self):
        return {"log2_M": self.log2_M, "log2_m": self.log2_m, "u": self.u, "p_bits": self.p_bits,
                "z": self.z, "radices": [self.radix_log2[i] for i in range(self.n_levels)],
                "cutoff_bits": self.cutoff_bits}


class SmulParams(ctypes.Structure):
    """dkss_smul_params: FFT length 2^log2_n and K = 2048 lw (0: the library's choice); s, K and
    n_levels are filled in by smul_select."""
    _fields_ = [("log2_n", ctypes.c_uint32), ("lw", ctypes.c_uint32), ("s", ctypes.c_uint32),
                ("K", ctypes.c_uint32), ("n_levels", ctypes.c_uint32), ("products", ctypes.c_uint32)]

    @classmethod
    def make(cls, log2_n=0, lw=0, products=0):
        p = cls()
        p.log2_n, p.lw, p.products = log2_n, lw, products
        return p

    def as_dict(self):
        return {"log2_n": self.log2_n, "lw": self.lw, "s": self.s, "K": self.K,
                "n_levels": self.n_levels, "products": self.products}


class Plan(ctypes.Structure):
    _fields_ = [("params", Params), ("L", ctypes.c_uint32), ("q_bits", ctypes.c_uint32),
                ("schoolbook", ctypes.c_uint32), ("squaring", ctypes.c_uint32),
                ("poly_bytes", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64),
                ("q", ctypes.c_uint32 * 16), ("digits", ctypes.c_uint32)]

    @property
    def modulus(self):
        return sum(int(self.q[i]) << (32 * i) for i in range(self.L))


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("alg_ops", ctypes.c_double)]


KERNEL_KINDS = 11

_lib = None


def lib():
    """Load libdkss.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdkss.so is not built: run python -m paper_1503_04955_amd.build")
        # One HIP runtime per process: torch ships its own libamdhip64 (same soname), so torch is
        # loaded first and the library binds to that copy.  Loaded the other way round, the
        # process would hold two runtimes and the second would find no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, u32, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint64
        PP = ctypes.POINTER(Params)
        L.dkss_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_char_p]
        L.dkss_ctx_destroy.argtypes = [vp]
        L.dkss_ctx_destroy.restype = None
        L.dkss_select_params.argtypes = [vp, u64, u64, u32, PP]
        L.dkss_plan_info.argtypes = [vp, sz, sz, PP, ctypes.POINTER(Plan)]
        L.dkss_workspace_bytes.argtypes = [vp, sz, sz, PP, ctypes.POINTER(sz)]
        L.dkss_prepare.argtypes = [vp, sz, sz, PP, vp]
        L.dkss_mul.argtypes = [vp, vp, vp, sz, vp, sz, PP, vp, sz, vp]
        L.dkss_mul_noalloc.argtypes = [vp, vp, vp, sz, vp, sz, PP, vp]
        L.dkss_probe_mad_rate.argtypes = [ctypes.POINTER(ctypes.c_double), vp]
        L.dkss_probe_twiddle_products.argtypes = [ctypes.c_int, ctypes.POINTER(u32), u32, u32, sz, vp, vp,
                                                  vp, vp, vp]
        SP = ctypes.POINTER(SmulParams)
        L.dkss_smul_select.argtypes = [sz, sz, SP]
        L.dkss_smul_workspace_bytes.argtypes = [sz, sz, SP, ctypes.POINTER(sz)]
        L.dkss_smul.argtypes = [vp, vp, sz, vp, sz, SP, vp, sz, vp]
        L.dkss_smul_forward.argtypes = [vp, vp, vp, sz, sz, SP, vp]
        L.dkss_mul_batch.argtypes = [vp, sz, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(sz), ctypes.POINTER(vp), ctypes.POINTER(sz), PP,
                                     vp, sz, vp]
        L.dkss_batch_workspace_bytes.argtypes = [vp, sz, ctypes.POINTER(sz), ctypes.POINTER(sz), PP,
                                                 ctypes.POINTER(sz)]
        L.dkss_batch_prepare.argtypes = [vp, sz, ctypes.POINTER(sz), ctypes.POINTER(sz), PP, vp]
        L.dkss_forward.argtypes = [vp, vp, vp, sz, sz, PP, vp, sz, vp]
        L.dkss_residues.argtypes = [vp, sz, ctypes.POINTER(u64), sz, vp, vp]
        L.dkss_profile_enable.argtypes = [vp, ctypes.c_int]
        L.dkss_profile_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(KernelStats)]
        L.dkss_profile_reset.argtypes = [vp]
        L.dkss_kernel_name.argtypes = [ctypes.c_int]
        L.dkss_kernel_name.restype = ctypes.c_char_p
        L.dkss_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_longlong]
        L.dkss_candidates.argtypes = [vp, u64, u64, PP, ctypes.POINTER(ctypes.c_int)]
        fp = ctypes.POINTER(ctypes.c_float)
        L.dkss_mlp_features.argtypes = [u64, u64, u32, fp]
        L.dkss_mlp_forward.argtypes = [vp, vp, ctypes.c_int, vp, vp]
        L.dkss_mlp_work_floats.argtypes = [ctypes.c_int]
        L.dkss_mlp_work_floats.restype = sz
        L.dkss_mlp_loss_grad.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, vp, vp, vp, vp]
        L.dkss_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, vp]
        L.dkss_set_mlp.argtypes = [vp, fp]
        L.dkss_mlp_load.argtypes = [ctypes.c_char_p, fp]
        L.dkss_mlp_choose.argtypes = [vp, u64, u64, u32, ctypes.POINTER(ctypes.c_int)]
        L.dkss_batch_graph_create.argtypes = [vp, sz, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(sz), ctypes.POINTER(vp),
                                              ctypes.POINTER(sz), PP, vp, sz, ctypes.POINTER(vp)]
        L.dkss_graph_launch.argtypes = [vp, vp]
        L.dkss_graph_info.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.dkss_graph_destroy.argtypes = [vp]
        L.dkss_graph_destroy.restype = None
        L.dkss_last_hip_error.argtypes = []
        L.dkss_hip_error_string.argtypes = [ctypes.c_int]
        L.dkss_hip_error_string.restype = ctypes.c_char_p
        L.dkss_strerror.argtypes = [ctypes.c_int]
        L.dkss_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ["dkss_ctx_create", "dkss_ctx_destroy", "dkss_select_params", "dkss_plan_info",
            "dkss_workspace_bytes", "dkss_prepare", "dkss_mul", "dkss_mul_noalloc", "dkss_mul_batch",
            "dkss_smul_select", "dkss_smul_workspace_bytes", "dkss_smul", "dkss_smul_forward",
            "dkss_probe_mad_rate", "dkss_probe_twiddle_products",
            "dkss_batch_workspace_bytes", "dkss_batch_prepare", "dkss_forward", "dkss_residues", "dkss_profile_enable",
            "dkss_profile_read", "dkss_profile_reset", "dkss_kernel_name", "dkss_set_option",
            "dkss_candidates", "dkss_mlp_features", "dkss_mlp_forward", "dkss_mlp_work_floats",
            "dkss_mlp_loss_grad", "dkss_mlp_adam", "dkss_set_mlp", "dkss_mlp_load",
            "dkss_mlp_choose", "dkss_batch_graph_create", "dkss_graph_launch", "dkss_graph_info",
            "dkss_graph_destroy", "dkss_last_hip_error", "dkss_hip_error_string", "dkss_strerror"]

NCAND = 24
MLP_IN, MLP_HID, MLP_OUT = 3, 64, NCAND + 1
CAND_SCHOOLBOOK = NCAND
MLP_NPARAM = MLP_HID * MLP_IN + MLP_HID + MLP_HID * MLP_HID + MLP_HID + MLP_OUT * MLP_HID + MLP_OUT
TUNING_DIR = os.path.join(_HERE, "tuning")

OPT_OVERLAP, OPT_DFT_LDS, OPT_FUSE_PW, OPT_BATCH_LANES, OPT_STEP6_KS = 0, 1, 2, 3, 4


def _check(rc, what):
    if rc != OK:
        raise DkssError(rc, what)


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _check_limbs(name, t, device=None):
    """An integer argument: a contiguous torch.int32 tensor on the device (a strided view or
    another dtype would be read as the wrong limbs)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.int32:
        raise TypeError("%s must be torch.int32 (uint32 limbs), not %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if not t.is_cuda or (device is not None and t.device != device):
        raise ValueError("%s must be on device %s" % (name, device if device is not None else "cuda"))


def _capturing():
    torch = _torch()
    return torch.cuda.is_available() and torch.cuda.is_current_stream_capturing()


def _keep_until_done(stream, *tensors):
    """Tensors allocated on the current stream and used by work on another stream stay
    allocated until that work is done."""
    if stream is None:
        return
    torch = _torch()
    if stream == torch.cuda.current_stream():
        return
    for t in tensors:
        if t is not None and t.numel():
            t.record_stream(stream)


def _pp(params):
    return ctypes.byref(params) if params is not None else None


def probe_mad_rate(stream=None):
    """Measured v_mad_u64_u32 lane operations per second on the current device."""
    r = ctypes.c_double()
    _check(lib().dkss_probe_mad_rate(ctypes.byref(r), _stream_ptr(stream)), "dkss_probe_mad_rate")
    return r.value


def probe_twiddle_products(form, q, L, groups, t, x, r, y, log2_m=4, stream=None):
    """dkss_probe_twiddle_products: y[g][n] = t[g] alpha^r[g][n] x[g][n] 2^(-28K) mod q for groups of
    32 elements sharing one twiddle; form 1 vector units, 2 matrix cores.  q: an int; t, x, r, y:
    int32 device tensors (groups x m x L, groups x 32 x m x L, groups x 32, as x)."""
    qa = (ctypes.c_uint32 * L)(*[(q >> (32 * k)) & 0xFFFFFFFF for k in range(L)])
    _check(lib().dkss_probe_twiddle_products(form, qa, L, log2_m, groups, _ptr(t), _ptr(x), _ptr(r),
                                             _ptr(y), _stream_ptr(stream)),
           "dkss_probe_twiddle_products")


def smul_select(alen, blen):
    """The library's SMUL parameters for alen x blen limbs (dkss_smul_select)."""
    p = SmulParams()
    _check(lib().dkss_smul_select(alen, blen, ctypes.byref(p)), "dkss_smul_select")
    return p


def smul_workspace_bytes(alen, blen, params=None):
    n = ctypes.c_size_t()
    _check(lib().dkss_smul_workspace_bytes(alen, blen, _pp(params), ctypes.byref(n)),
           "dkss_smul_workspace_bytes")
    return n.value


def smul(a, b, out=None, params=None, ws=None, stream=None):
    """c = a * b by Schoenhage-Strassen multiplication (dkss_smul) for int32 (uint32-limb)
    device tensors; returns c (alen + blen limbs)."""
    torch = _torch()
    _check_limbs("a", a)
    _check_limbs("b", b, a.device)
    alen, blen = a.numel(), b.numel()
    if out is None:
        out = torch.empty(alen + blen, dtype=torch.int32, device=a.device)
    _check_limbs("out", out, a.device)
    if out.numel() < alen + blen:
        raise ValueError("out holds %d limbs, the product %d" % (out.numel(), alen + blen))
    if ws is None:
        ws = _alloc_ws(smul_workspace_bytes(alen, blen, params), a.device)
    _check(lib().dkss_smul(_ptr(out), _ptr(a), alen, _ptr(b), blen, _pp(params), _ptr(ws), ws.numel(),
                           _stream_ptr(stream)), "dkss_smul")
    _keep_until_done(stream, ws, out)
    return out


def smul_forward(a, alen, blen, params=None, stream=None):
    """SMUL's forward transform of a for an alen x blen product (dkss_smul_forward): returns
    (poly, tops) in bit-reversed order, poly as (n, 64 lw) int32 limbs, tops (n,) int32."""
    torch = _torch()
    _check_limbs("a", a)
    p = SmulParams()
    if params is not None:
        p.log2_n, p.lw = params.log2_n, params.lw
    _check(lib().dkss_smul_select(alen, blen, ctypes.byref(p)) if params is None else OK, "dkss_smul_select")
    n, W = 1 << p.log2_n, 64 * p.lw
    poly = torch.empty((n, W), dtype=torch.int32, device=a.device)
    tops = torch.empty(n, dtype=torch.int32, device=a.device)
    _check(lib().dkss_smul_forward(_ptr(poly), _ptr(tops), _ptr(a), alen, blen, ctypes.byref(p),
                                   _stream_ptr(stream)), "dkss_smul_forward")
    return poly, tops


def to_device(limbs, device="cuda"):
    """numpy uint32 limbs -> torch.int32 device tensor (same bits)."""
    torch = _torch()
    arr = np.ascontiguousarray(limbs, dtype=np.uint32).view(np.int32)
    return torch.from_numpy(arr.copy()).to(device)


def to_host(t):
    """torch.int32 device tensor -> numpy uint32 limbs."""
    return t.detach().cpu().numpy().view(np.uint32)


def _alloc_ws(nbytes, device):
    torch = _torch()
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


class Context:
    """A libdkss context: cached parameter constants and device tables."""

    def __init__(self, policy=POLICY_THESIS, tuning_dir=None):
        """policy POLICY_THESIS (the thesis's rule), POLICY_TUNED (the measured table in
        tuning_dir/dkss_tuning.txt) or POLICY_LEARNED (the selector weights in
        tuning_dir/dkss_mlp.txt); tuning_dir defaults to the package's tuning folder; without
        the file the policy falls back to the thesis's rule."""
        h = ctypes.c_void_p()
        d = tuning_dir if tuning_dir is not None else TUNING_DIR
        _check(lib().dkss_ctx_create(ctypes.byref(h), policy, d.encode()), "dkss_ctx_create")
        self._h = h
        self._prepared = set()

    def close(self):
        if self._h:
            lib().dkss_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def select_params(self, a_bits, b_bits, batch=1):
        p = Params()
        _check(lib().dkss_select_params(self._h, a_bits, b_bits, batch, ctypes.byref(p)),
               "dkss_select_params")
        return p

    def candidates(self, a_bits, b_bits):
        """[(index, Params)] of the feasible candidate tuples for these operand sizes."""
        arr = (Params * NCAND)()
        valid = (ctypes.c_int * NCAND)()
        _check(lib().dkss_candidates(self._h, a_bits, b_bits, arr, valid), "dkss_candidates")
        return [(c, arr[c]) for c in range(NCAND) if valid[c]]

    def plan_info(self, alen, blen, params=None):
        out = Plan()
        _check(lib().dkss_plan_info(self._h, alen, blen, _pp(params), ctypes.byref(out)),
               "dkss_plan_info")
        return out

    def workspace_bytes(self, alen, blen, params=None):
        n = ctypes.c_size_t()
        _check(lib().dkss_workspace_bytes(self._h, alen, blen, _pp(params), ctypes.byref(n)),
               "dkss_workspace_bytes")
        return n.value

    def prepare(self, alen, blen, params=None, stream=None):
        """Build the tuple's table in the context (dkss_prepare: allocates, waits)."""
        _check(lib().dkss_prepare(self._h, alen, blen, _pp(params), _stream_ptr(stream)),
               "dkss_prepare")
        self._prepared.add((alen, blen, bytes(params) if params is not None else None))

    def mul(self, a, b, out=None, params=None, ws=None, stream=None, prepare=True):
        """c = a * b for int32 (uint32-limb) device tensors; returns c (alen+blen limbs).
        prepare: on the first product of a shape outside a stream capture, dkss_prepare builds
        the tuple's table in the context (otherwise every call builds it in its workspace)."""
        torch = _torch()
        _check_limbs("a", a)
        _check_limbs("b", b, a.device)
        alen, blen = a.numel(), b.numel()
        if out is None:
            out = torch.empty(alen + blen, dtype=torch.int32, device=a.device)
        _check_limbs("out", out, a.device)
        if out.numel() < alen + blen:
            raise ValueError("out holds %d limbs, the product %d" % (out.numel(), alen + blen))
        key = (alen, blen, bytes(params) if params is not None else None)
        if prepare and key not in self._prepared and not _capturing():
            self.prepare(alen, blen, params, stream)
        if ws is None:
            ws = _alloc_ws(self.workspace_bytes(alen, blen, params), a.device)
        _check(lib().dkss_mul(self._h, _ptr(out), _ptr(a), alen, _ptr(b), blen, _pp(params),
                              _ptr(ws), ws.numel(), _stream_ptr(stream)), "dkss_mul")
        _keep_until_done(stream, ws, out)
        return out

    def mul_noalloc(self, a, b, out, params=None, stream=None):
        """out = a * b through dkss_mul_noalloc: no workspace, no preparation, no allocation
        (the library's fixed scratch on the current device; out is the caller's tensor)."""
        _check_limbs("a", a)
        _check_limbs("b", b, a.device)
        _check_limbs("out", out, a.device)
        alen, blen = a.numel(), b.numel()
        if out.numel() < alen + blen:
            raise ValueError("out holds %d limbs, the product %d" % (out.numel(), alen + blen))
        _check(lib().dkss_mul_noalloc(self._h, _ptr(out), _ptr(a), alen, _ptr(b), blen, _pp(params),
                                      _stream_ptr(stream)), "dkss_mul_noalloc")
        return out

    def mul_batch(self, as_, bs, outs=None, params=None, ws=None, stream=None):
        """outs[i] = as_[i] * bs[i] in one dkss_mul_batch call; returns outs."""
        call = BatchCall(self, as_, bs, outs, params, ws)
        call(stream)
        return call.outs

    def set_mlp(self, weights):
        """Install selector weights (MLP_NPARAM floats) for POLICY_LEARNED; None removes them."""
        if weights is None:
            _check(lib().dkss_set_mlp(self._h, None), "dkss_set_mlp")
            return
        w = np.ascontiguousarray(weights, dtype=np.float32)
        assert w.size == MLP_NPARAM
        _check(lib().dkss_set_mlp(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "dkss_set_mlp")

    def mlp_choose(self, a_bits, b_bits, batch=1):
        """The selector's choice: a candidate index, CAND_SCHOOLBOOK, or -1 (thesis rule)."""
        c = ctypes.c_int()
        _check(lib().dkss_mlp_choose(self._h, a_bits, b_bits, batch, ctypes.byref(c)),
               "dkss_mlp_choose")
        return c.value

    def set_option(self, option, value):
        _check(lib().dkss_set_option(self._h, option, int(value)), "dkss_set_option")

    def profile(self, on=True):
        _check(lib().dkss_profile_enable(self._h, 1 if on else 0), "dkss_profile_enable")

    def profile_reset(self):
        _check(lib().dkss_profile_reset(self._h), "dkss_profile_reset")

    def profile_read(self):
        """{kernel name: KernelStats} for every kind launched since the last reset."""
        out = {}
        for k in range(KERNEL_KINDS):
            st = KernelStats()
            _check(lib().dkss_profile_read(self._h, k, ctypes.byref(st)), "dkss_profile_read")
            if st.launches:
                out[lib().dkss_kernel_name(k).decode()] = st
        return out

    def forward(self, a, blen, params=None, stream=None):
        """encode + forward transform of a (operand pair a x blen limbs); natural order."""
        torch = _torch()
        _check_limbs("a", a)
        plan = self.plan_info(a.numel(), blen, params)
        poly = torch.empty(plan.poly_bytes // 4, dtype=torch.int32, device=a.device)
        ws = _alloc_ws(self.workspace_bytes(a.numel(), blen, params), a.device)
        _check(lib().dkss_forward(self._h, _ptr(poly), _ptr(a), a.numel(), blen, _pp(params),
                                  _ptr(ws), ws.numel(), _stream_ptr(stream)), "dkss_forward")
        return poly


class BatchCall:
    """A dkss_mul_batch call with its arguments marshalled once, for repeated launches over the
    same tensors (the products are recomputed by every call)."""

    def __init__(self, ctx, as_, bs, outs=None, params=None, ws=None, alloc_ws=True, prepare=True):
        torch = _torch()
        n = len(as_)
        if len(bs) != n or (outs is not None and len(outs) != n):
            raise ValueError("as_, bs and outs must have the same length")
        dev = as_[0].device if n else None
        for i in range(n):
            _check_limbs("as_[%d]" % i, as_[i], dev)
            _check_limbs("bs[%d]" % i, bs[i], dev)
        if outs is None:
            outs = [torch.empty(a.numel() + b.numel(), dtype=torch.int32, device=a.device)
                    for a, b in zip(as_, bs)]
        for i, (o, a, b) in enumerate(zip(outs, as_, bs)):
            _check_limbs("outs[%d]" % i, o, dev)
            if o.numel() < a.numel() + b.numel():
                raise ValueError("outs[%d] is too short" % i)
        self.ctx, self.as_, self.bs, self.outs, self.n = ctx, as_, bs, outs, n
        VP = ctypes.c_void_p * n
        SZ = ctypes.c_size_t * n
        self.al = SZ(*[a.numel() for a in as_])
        self.bl = SZ(*[b.numel() for b in bs])
        self.pa = (Params * n)(*params) if params is not None else None
        self.pc = VP(*[_ptr(o) for o in outs])
        self.pa_ptrs = VP(*[_ptr(a) for a in as_])
        self.pb_ptrs = VP(*[_ptr(b) for b in bs])
        nb = ctypes.c_size_t()
        _check(lib().dkss_batch_workspace_bytes(ctx._h, n, self.al, self.bl, self.pa,
                                                ctypes.byref(nb)), "dkss_batch_workspace_bytes")
        self.ws_bytes = nb.value
        if prepare and n and not _capturing():
            _check(lib().dkss_batch_prepare(ctx._h, n, self.al, self.bl, self.pa, _stream_ptr(None)),
                   "dkss_batch_prepare")
        if ws is None and alloc_ws:
            ws = _alloc_ws(nb.value, as_[0].device)
        self.ws = ws

    def __call__(self, stream=None):
        _check(lib().dkss_mul_batch(self.ctx._h, self.n, self.pc, self.pa_ptrs, self.al,
                                    self.pb_ptrs, self.bl, self.pa, _ptr(self.ws),
                                    self.ws.numel(), _stream_ptr(stream)), "dkss_mul_batch")
        _keep_until_done(stream, self.ws, *self.outs)
        return self.outs

    def graph(self):
        """Capture this batch into a HIP graph (BatchGraph); it uses this call's workspace."""
        return BatchGraph(self)


class BatchGraph:
    """A batch captured once (dkss_batch_graph_create) and replayed with one graph launch."""

    def __init__(self, call):
        h = ctypes.c_void_p()
        _check(lib().dkss_batch_graph_create(call.ctx._h, call.n, call.pc, call.pa_ptrs, call.al,
                                             call.pb_ptrs, call.bl, call.pa, _ptr(call.ws),
                                             call.ws.numel(), ctypes.byref(h)),
               "dkss_batch_graph_create")
        self._h = h
        self.call = call                     # keeps buffers and the context alive
        n, k = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().dkss_graph_info(h, ctypes.byref(n), ctypes.byref(k)), "dkss_graph_info")
        self.products, self.kernels = n.value, k.value

    def __call__(self, stream=None):
        _check(lib().dkss_graph_launch(self._h, _stream_ptr(stream)), "dkss_graph_launch")
        return self.call.outs

    def close(self):
        if self._h:
            _torch().cuda.synchronize()
            lib().dkss_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def residues(x, primes, stream=None):
    """x mod q for each q in primes (odd, < 2^62), computed on the device."""
    torch = _torch()
    out = torch.empty(len(primes), dtype=torch.int64, device=x.device)
    arr = (ctypes.c_uint64 * len(primes))(*primes)
    _check(lib().dkss_residues(_ptr(x), x.numel(), arr, len(primes), _ptr(out),
                               _stream_ptr(stream)), "dkss_residues")
    return [int(v) & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]


# ----- learned selector: the network's kernels ------------------------------------------------

def mlp_features(a_bits, b_bits, batch=1):
    """The selector's inputs for one product (numpy float32[MLP_IN])."""
    out = (ctypes.c_float * MLP_IN)()
    _check(lib().dkss_mlp_features(a_bits, b_bits, batch, out), "dkss_mlp_features")
    return np.array(out[:], dtype=np.float32)


def mlp_load(path):
    """Selector weights from a text file (numpy float32[MLP_NPARAM])."""
    w = np.zeros(MLP_NPARAM, dtype=np.float32)
    _check(lib().dkss_mlp_load(path.encode(), w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
           "dkss_mlp_load")
    return w


def mlp_save(path, weights, comment=""):
    """Write weights in the text form dkss_mlp_load reads."""
    w = np.asarray(weights, dtype=np.float32).ravel()
    assert w.size == MLP_NPARAM
    with open(path, "w") as f:
        for line in comment.splitlines():
            f.write("# %s\n" % line)
        f.write("%d %d %d\n" % (MLP_IN, MLP_HID, MLP_OUT))
        for v in w:
            f.write("%.9g\n" % float(v))


def mlp_forward(params, x, y=None, stream=None):
    """y[n][MLP_OUT] = network(x[n][MLP_IN]); float32 device tensors."""
    torch = _torch()
    n = x.shape[0]
    if y is None:
        y = torch.empty((n, MLP_OUT), dtype=torch.float32, device=x.device)
    _check(lib().dkss_mlp_forward(_ptr(params), _ptr(x), n, _ptr(y), _stream_ptr(stream)),
           "dkss_mlp_forward")
    return y


def mlp_work(n, device="cuda"):
    """A work buffer for mlp_loss_grad over n samples."""
    torch = _torch()
    return torch.empty(lib().dkss_mlp_work_floats(n), dtype=torch.float32, device=device)


def mlp_loss_grad(params, x, t, mask, mask_sum, grad=None, loss=None, work=None, stream=None):
    """(grad[MLP_NPARAM], loss[1]) of the masked squared error; float32 device tensors."""
    torch = _torch()
    n = x.shape[0]
    if grad is None:
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    if work is None:
        work = mlp_work(n, x.device)
    _check(lib().dkss_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(t), _ptr(mask), n,
                                    float(mask_sum), _ptr(grad), _ptr(loss), _ptr(work),
                                    _stream_ptr(stream)), "dkss_mlp_loss_grad")
    return grad, loss


def mlp_adam(params, grad, m1, m2, step, lr, stream=None):
    """One Adam step in place on float32 device tensors (step counts from 1)."""
    _check(lib().dkss_mlp_adam(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(step), float(lr),
                               _stream_ptr(stream)), "dkss_mlp_adam")
