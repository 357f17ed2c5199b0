"""Python binding of libpdfmi.so (include/pdfmi.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; torch is used
for device memory and streams.  torch is imported before the library is
loaded so that both share one HIP runtime.  If the library has not been built,
importing this module raises: there is no fallback implementation.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdfmi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libpdfmi.so is not built (run __graft_entry__.build() or "
                      "python paper_2009_06635_amd/build.py); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64
_SIGS = {
    "pdf_load_grid": [_i32, _P, _i32, _P, _P, _P, _P],
    "pdf_unload": [_i32],
    "pdf_load_alphas": [_i32, _P, _P],
    "pdf_xfxq2": [_i32, _P, _i32, _P, _P, _i64, _P, _P],
    "pdf_xfxq2_f32": [_i32, _P, _i32, _P, _P, _i64, _P, _P],
    "pdf_alphas_q2": [_P, _i64, _P, _P],
    "pdf_locate": [_i32, _P, _P, _i64, _P, _P, _P, _P, _P],
    "pdf_error_count": [_P, _i32, _P],
    "pdf_validate_grid": [_i32, _P, _i32, _P, _P, _P],
    "pdf_validate_alphas": [_i32, _P, _P],
    "pdf_set_lds_policy": [_i32],
    "pdf_set_tuning": [_i32, _i32],
    "pdf_get_tuning": [_i32, _P],
    "pdf_mc_workspace_bytes": [_i64, _P],
    "pdf_mc_chunk_sum": [_P, _P, _i32, _P, _i64, _P, _P, _P],
    "pdf_mc_chunk_sum_f32": [_P, _P, _i32, _P, _i64, _P, _P, _P],
    "pdf_batch_create": [_P, _i32, _i32, _P],
    "pdf_batch_configure": [_i32, _i32, _i32, _i32],
    "pdf_batch_run": [_i32, _P],
    "pdf_batch_autotune": [_i32, _i32, _P, _P, _P],
    "pdf_batch_tune_cache": [ctypes.c_char_p],
    "pdf_batch_destroy": [_i32],
    "pdf_xfxq2_batched": [_P, _i32, _P],
    "pdf_xfxq2_batched_f64": [_P, _i32, _P],
    "pdf_surrogate_param_count": [_P],
    "pdf_surrogate_create": [_i32, ctypes.c_uint64, _P],
    "pdf_surrogate_destroy": [_i32],
    "pdf_surrogate_set_data": [_i32, _P, _P, _i64, _P],
    "pdf_surrogate_train": [_i32, _P, _P],
    "pdf_surrogate_adam": [_i32, _P, ctypes.c_float, _P],
    "pdf_surrogate_grad": [_i32, _P, _P, _i32, _P, _P, _P],
    "pdf_surrogate_params": [_i32, _P, _i32],
    "pdf_surrogate_xfxq2": [_i32, _P, _i32, _P, _P, _i64, _P, _P],
    "pdf_surrogate_save": [_i32, ctypes.c_char_p],
    "pdf_surrogate_load": [_i32, ctypes.c_char_p],
    "pdf_shutdown": [],
    "pdf_xfxq2_alphas": [_i32, _P, _i32, _P, _P, _i64, _P, _P, _P],
    "pdf_xfxq2_alphas_f32": [_i32, _P, _i32, _P, _P, _i64, _P, _P, _P],
    "pdf_mc_fused": [_i32, _P, _i32, _P, _P, _P, _i64, _P, _P, _P],
    "pdf_mc_fused_f32": [_i32, _P, _i32, _P, _P, _P, _i64, _P, _P, _P],
    "pdf_fk_contract": [_P, _P, _i32, _i32, _i64, _P, _P],
    "pdf_fk_contract_noalloc": [_P, _P, _i32, _i32, _i64, _P, _P],
    "pdf_lhapdf_read": [ctypes.c_char_p, _P, _P, _P, _P, _P],
    "pdf_load_lhapdf": [ctypes.c_char_p, _P],
    "pdf_lhapdf_read_alphas": [ctypes.c_char_p, _P, _P, _P],
    "pdf_load_lhapdf_alphas": [ctypes.c_char_p],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.pdf_last_error.argtypes = []
_lib.pdf_last_error.restype = ctypes.c_char_p

PDF_OK, PDF_ERR_ARG, PDF_ERR_GRID, PDF_ERR_MEMBER, PDF_ERR_PID, PDF_ERR_NOMEM, PDF_ERR_DEVICE, PDF_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7


class PdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pdfmi error %d: %s" % (code, msg))
        self.code = code


def library():
    """The loaded ctypes library (for ABI-level tests)."""
    return _lib


def last_error():
    return _lib.pdf_last_error().decode()


def _check(rc):
    if rc != PDF_OK:
        raise PdfError(rc, last_error())


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(_P)


def _grid_arrays(xknots, q2knots, values, pids):
    shape = _np([[len(x), len(q)] for x, q in zip(xknots, q2knots)], np.int32)
    knots = _np(np.concatenate([np.concatenate([np.asarray(x, np.float64), np.asarray(q, np.float64)])
                                for x, q in zip(xknots, q2knots)]), np.float64)
    vals = _np(np.concatenate([np.asarray(v, np.float64).ravel() for v in values]), np.float64)
    return shape, _np(pids, np.int32), knots, vals


def validate_grid(xknots, q2knots, values, pids):
    """Host-only grid check; returns the status code (no GPU needed)."""
    shape, p, knots, vals = _grid_arrays(xknots, q2knots, values, pids)
    return _lib.pdf_validate_grid(len(shape), _ptr(shape), len(p), _ptr(p), _ptr(knots), _ptr(vals))


def validate_alphas(q2knots, alphas):
    k, a = _np(q2knots, np.float64), _np(alphas, np.float64)
    return _lib.pdf_validate_alphas(len(k), _ptr(k), _ptr(a))


def load_grid(xknots, q2knots, values, pids):
    """Copy one member's grid to the device; returns the member id."""
    shape, p, knots, vals = _grid_arrays(xknots, q2knots, values, pids)
    mid = ctypes.c_int32(-1)
    _check(_lib.pdf_load_grid(len(shape), _ptr(shape), len(p), _ptr(p), _ptr(knots), _ptr(vals),
                              ctypes.byref(mid)))
    return mid.value


def load_synth(grid):
    """Load a SynthGrid (paper_2009_06635_amd.synth)."""
    return load_grid(grid.xknots, grid.q2knots, grid.values, grid.pids)


def unload(member):
    _check(_lib.pdf_unload(int(member)))


def load_alphas(q2knots, alphas):
    k, a = _np(q2knots, np.float64), _np(alphas, np.float64)
    _check(_lib.pdf_load_alphas(len(k), _ptr(k), _ptr(a)))


def read_lhapdf(path):
    """Parse an LHAPDF6 member file (lhagrid1) on the host: returns
    (xknots, q2knots, values, pids) per sub-grid, Q knots squared."""
    sizes = np.zeros(4, np.int64)
    bpath = str(path).encode()
    _check(_lib.pdf_lhapdf_read(bpath, _ptr(sizes), None, None, None, None))
    K, P, nk, nv = (int(v) for v in sizes)
    shape = np.zeros(2 * K, np.int32)
    pids = np.zeros(P, np.int32)
    knots = np.zeros(nk, np.float64)
    vals = np.zeros(nv, np.float64)
    _check(_lib.pdf_lhapdf_read(bpath, _ptr(sizes), _ptr(shape), _ptr(pids), _ptr(knots), _ptr(vals)))
    xk, qk, vs = [], [], []
    ko = vo = 0
    for k in range(K):
        nx, nq = int(shape[2 * k]), int(shape[2 * k + 1])
        xk.append(knots[ko:ko + nx].copy())
        qk.append(knots[ko + nx:ko + nx + nq].copy())
        vs.append(vals[vo:vo + nx * nq * P].reshape(nx, nq, P).copy())
        ko += nx + nq
        vo += nx * nq * P
    return xk, qk, vs, pids.tolist()


def load_lhapdf(path):
    """Read an LHAPDF6 member file and load it; returns the member id."""
    mid = ctypes.c_int32(-1)
    _check(_lib.pdf_load_lhapdf(str(path).encode(), ctypes.byref(mid)))
    return mid.value


def read_lhapdf_alphas(info_path):
    """(Q^2 knots, alpha_s values) of a set's .info file."""
    n = ctypes.c_int32(0)
    bpath = str(info_path).encode()
    _check(_lib.pdf_lhapdf_read_alphas(bpath, ctypes.byref(n), None, None))
    q2 = np.zeros(n.value, np.float64)
    a = np.zeros(n.value, np.float64)
    _check(_lib.pdf_lhapdf_read_alphas(bpath, ctypes.byref(n), _ptr(q2), _ptr(a)))
    return q2, a


def load_lhapdf_alphas(info_path):
    _check(_lib.pdf_load_lhapdf_alphas(str(info_path).encode()))


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return _P(s.cuda_stream)


def _dev_f64(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("%s must be a contiguous float64 CUDA tensor" % name)
    return t


def _pid_arg(pids):
    if pids is None:
        return None, 0
    arr = _np(pids, np.int32)
    return arr, len(arr)


def n_columns(member_pids, pids):
    return len(member_pids) if pids is None else len(pids)


def xfxq2(member, pids, x, q2, out=None, n_cols=None, stream=None):
    """x*f, FP64, point-major [n][len(pids)] (pids=None: every stored column,
    then pass n_cols = number of stored columns)."""
    _dev_f64(x, "x")
    _dev_f64(q2, "q2")
    arr, npid = _pid_arg(pids)
    cols = npid if pids is not None else n_cols
    if out is None:
        out = torch.empty((x.shape[0], cols), dtype=torch.float64, device=x.device)
    _check(_lib.pdf_xfxq2(int(member), _ptr(arr) if arr is not None else None, npid, _P(x.data_ptr()),
                          _P(q2.data_ptr()), x.shape[0], _P(out.data_ptr()), _stream(stream)))
    return out


def xfxq2_alphas(member, pids, x, q2, out=None, alphas_out=None, f32=False, n_cols=None, stream=None):
    """x*f (FP64, or FP32 arithmetic with f32) and alpha_s at the same points
    in one pass; returns (out, alphas_out)."""
    _dev_f64(x, "x")
    _dev_f64(q2, "q2")
    arr, npid = _pid_arg(pids)
    cols = npid if pids is not None else n_cols
    if out is None:
        out = torch.empty((x.shape[0], cols), dtype=torch.float32 if f32 else torch.float64, device=x.device)
    if alphas_out is None:
        alphas_out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    fn = _lib.pdf_xfxq2_alphas_f32 if f32 else _lib.pdf_xfxq2_alphas
    _check(fn(int(member), _ptr(arr) if arr is not None else None, npid, _P(x.data_ptr()), _P(q2.data_ptr()),
              x.shape[0], _P(out.data_ptr()), _P(alphas_out.data_ptr()), _stream(stream)))
    return out, alphas_out


def xfxq2_f32(member, pids, x, q2, out=None, n_cols=None, stream=None):
    """x*f with FP32 bulk arithmetic; FP32 point-major output."""
    _dev_f64(x, "x")
    _dev_f64(q2, "q2")
    arr, npid = _pid_arg(pids)
    cols = npid if pids is not None else n_cols
    if out is None:
        out = torch.empty((x.shape[0], cols), dtype=torch.float32, device=x.device)
    _check(_lib.pdf_xfxq2_f32(int(member), _ptr(arr) if arr is not None else None, npid, _P(x.data_ptr()),
                              _P(q2.data_ptr()), x.shape[0], _P(out.data_ptr()), _stream(stream)))
    return out


def alphas_q2(q2, out=None, stream=None):
    _dev_f64(q2, "q2")
    if out is None:
        out = torch.empty_like(q2)
    _check(_lib.pdf_alphas_q2(_P(q2.data_ptr()), q2.shape[0], _P(out.data_ptr()), _stream(stream)))
    return out


def locate(member, x, q2, stream=None):
    """(subgrid, ix, iq, region) device tensors."""
    _dev_f64(x, "x")
    _dev_f64(q2, "q2")
    n = x.shape[0]
    k = torch.empty(n, dtype=torch.int32, device=x.device)
    ix = torch.empty_like(k)
    iq = torch.empty_like(k)
    reg = torch.empty(n, dtype=torch.int8, device=x.device)
    _check(_lib.pdf_locate(int(member), _P(x.data_ptr()), _P(q2.data_ptr()), n, _P(k.data_ptr()),
                           _P(ix.data_ptr()), _P(iq.data_ptr()), _P(reg.data_ptr()), _stream(stream)))
    return k, ix, iq, reg


def error_count(reset=False, stream=None):
    v = ctypes.c_int64(0)
    _check(_lib.pdf_error_count(ctypes.byref(v), 1 if reset else 0, _stream(stream)))
    return v.value


def mc_workspace(n, device="cuda"):
    v = ctypes.c_int64(0)
    _check(_lib.pdf_mc_workspace_bytes(int(n), ctypes.byref(v)))
    return torch.empty(max(1, v.value // 8), dtype=torch.float64, device=device)


def mc_chunk_sum(xf1, xf2, alphas, workspace=None, out=None, stream=None):
    """FP64 sum_i alphas[i] * sum_j xf1[i,j] * xf2[i,j] (fixed order); returns a
    one-element device tensor."""
    _dev_f64(alphas, "alphas")
    f32 = xf1.dtype == torch.float32
    for t in (xf1, xf2):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == xf1.dtype and t.dtype in (torch.float32, torch.float64)):
            raise TypeError("xf1, xf2 must be contiguous CUDA tensors of one float dtype")
    n, P = xf1.shape
    if workspace is None:
        workspace = mc_workspace(n, xf1.device)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=xf1.device)
    fn = _lib.pdf_mc_chunk_sum_f32 if f32 else _lib.pdf_mc_chunk_sum
    _check(fn(_P(xf1.data_ptr()), _P(xf2.data_ptr()), P, _P(alphas.data_ptr()), n, _P(workspace.data_ptr()),
              _P(out.data_ptr()), _stream(stream)))
    return out


def mc_fused(member, pids, x1, x2, q2, f32=False, workspace=None, out=None, stream=None):
    """The chunk sum of mc_chunk_sum(xfxq2(x1), xfxq2(x2), alphas_q2(q2)) in
    one kernel without materialising the PDF values (bit-identical result);
    f32 evaluates the PDFs as xfxq2_f32 does.  Returns a one-element device
    tensor."""
    for t, nm in ((x1, "x1"), (x2, "x2"), (q2, "q2")):
        _dev_f64(t, nm)
    n = x1.shape[0]
    if x2.shape[0] != n or q2.shape[0] != n:
        raise ValueError("x1, x2, q2 must have the same length")
    arr, npid = _pid_arg(pids)
    if workspace is None:
        workspace = mc_workspace(n, x1.device)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x1.device)
    fn = _lib.pdf_mc_fused_f32 if f32 else _lib.pdf_mc_fused
    _check(fn(int(member), _ptr(arr) if arr is not None else None, npid, _P(x1.data_ptr()), _P(x2.data_ptr()),
              _P(q2.data_ptr()), n, _P(workspace.data_ptr()), _P(out.data_ptr()), _stream(stream)))
    return out


def fk_contract(pdf, fk, out=None, stream=None, noalloc=False):
    """out[r][d] = sum_k pdf[r][k] fk[d][k] (FP64 matrix cores); pdf [nrep][K]
    and fk [ndat][K] contiguous float64 CUDA tensors (2-D, or more dimensions
    flattened after the first).  noalloc=True calls pdf_fk_contract_noalloc
    (partial sums in the library's fixed scratch array; out must be given)."""
    if noalloc and out is None:
        raise ValueError("noalloc needs a caller-provided out tensor")
    for t, nm in ((pdf, "pdf"), (fk, "fk")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("%s must be a contiguous float64 CUDA tensor" % nm)
    nrep, ndat = pdf.shape[0], fk.shape[0]
    K = pdf[0].numel() if nrep else (fk[0].numel() if ndat else 0)
    if (nrep and pdf[0].numel() != K) or (ndat and fk[0].numel() != K):
        raise ValueError("pdf and fk rows differ in length")
    if out is None:
        out = torch.empty((nrep, ndat), dtype=torch.float64, device=pdf.device)
    fn = _lib.pdf_fk_contract_noalloc if noalloc else _lib.pdf_fk_contract
    _check(fn(_P(pdf.data_ptr()), _P(fk.data_ptr()), nrep, ndat, K, _P(out.data_ptr()), _stream(stream)))
    return out


class _Request(ctypes.Structure):
    _fields_ = [("member", ctypes.c_int32), ("n_pids", ctypes.c_int32), ("pids", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("q2", ctypes.c_void_p), ("n", ctypes.c_int64), ("out", ctypes.c_void_p)]


def _request_array(requests, out_f64, keep):
    """ctypes array of pdf_request for [(member, pids, x, q2, out), ...]; the
    objects it points into are appended to keep."""
    arr = (_Request * max(1, len(requests)))()
    for i, (member, pids, x, q2, out) in enumerate(requests):
        _dev_f64(x, "x")
        _dev_f64(q2, "q2")
        want = torch.float64 if out_f64 else torch.float32
        if not (out.is_cuda and out.dtype == want and out.is_contiguous()):
            raise TypeError("out must be a contiguous %s CUDA tensor" % want)
        pa, npid = _pid_arg(pids)
        if pa is not None:
            keep.append(pa)
        keep.append((x, q2, out))
        arr[i] = _Request(int(member), npid, _ptr(pa) if pa is not None else None, x.data_ptr(),
                          q2.data_ptr(), x.shape[0], out.data_ptr())
    return arr


class BatchPlan:
    """A batched plan over requests [(member, pids, x, q2, out), ...] with
    device tensors x, q2 (float64) and out (float32, or float64 if out_f64)."""

    def __init__(self, requests, out_f64=False):
        self._keep = []
        arr = _request_array(requests, out_f64, self._keep)
        self._reqs = arr
        pid = ctypes.c_int32(-1)
        _check(_lib.pdf_batch_create(ctypes.cast(arr, _P), len(requests), 1 if out_f64 else 0, ctypes.byref(pid)))
        self.id = pid.value

    def configure(self, tile_points=4096, vector_cols=1, use_graph=0):
        _check(_lib.pdf_batch_configure(self.id, int(tile_points), int(vector_cols), int(use_graph)))

    def run(self, stream=None):
        _check(_lib.pdf_batch_run(self.id, _stream(stream)))

    def autotune(self, reps=3, stream=None):
        t, v = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.pdf_batch_autotune(self.id, int(reps), _stream(stream), ctypes.byref(t), ctypes.byref(v)))
        return t.value, v.value

    def destroy(self):
        if self.id >= 0:
            _check(_lib.pdf_batch_destroy(self.id))
            self.id = -1


def xfxq2_batched(requests, out_f64=False, stream=None):
    """One-shot batched evaluation (pdf_xfxq2_batched / pdf_xfxq2_batched_f64;
    synchronises the stream)."""
    keep = []
    arr = _request_array(requests, out_f64, keep)
    fn = _lib.pdf_xfxq2_batched_f64 if out_f64 else _lib.pdf_xfxq2_batched
    _check(fn(ctypes.cast(arr, _P), len(requests), _stream(stream)))


def surrogate_param_count():
    v = ctypes.c_int32(0)
    _check(_lib.pdf_surrogate_param_count(ctypes.byref(v)))
    return v.value


class _TrainOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("lr_final", ctypes.c_float), ("total_steps", ctypes.c_int32), ("loss_out", ctypes.c_void_p),
                ("use_graph", ctypes.c_int32)]


class Surrogate:
    """MLP surrogate of one member (see pdf_surrogate_* in include/pdfmi.h)."""

    def __init__(self, member, seed=0):
        sid = ctypes.c_int32(-1)
        _check(_lib.pdf_surrogate_create(int(member), ctypes.c_uint64(seed), ctypes.byref(sid)))
        self.id = sid.value
        self.n_params = surrogate_param_count()

    def set_data(self, x, q2, stream=None):
        _dev_f64(x, "x")
        _dev_f64(q2, "q2")
        _check(_lib.pdf_surrogate_set_data(self.id, _P(x.data_ptr()), _P(q2.data_ptr()), x.shape[0], _stream(stream)))

    def train(self, steps, batch, lr, lr_final, total_steps, loss_out=None, use_graph=True, stream=None):
        """steps Adam steps; loss_out: optional float32 CUDA tensor of >= steps
        entries receiving each step's batch loss; use_graph: replay one recorded
        graph per step (False: the same launches one by one)."""
        if loss_out is not None and not (isinstance(loss_out, torch.Tensor) and loss_out.is_cuda and
                                         loss_out.dtype == torch.float32 and loss_out.numel() >= steps):
            raise TypeError("loss_out must be a float32 CUDA tensor of at least `steps` entries")
        o = _TrainOpts(int(steps), int(batch), float(lr), float(lr_final), int(total_steps),
                       loss_out.data_ptr() if loss_out is not None else None, 1 if use_graph else 0)
        _check(_lib.pdf_surrogate_train(self.id, ctypes.byref(o), _stream(stream)))

    def adam(self, grad, lr, stream=None):
        """One Adam step with a float32 CUDA gradient of n_params entries."""
        if not (isinstance(grad, torch.Tensor) and grad.is_cuda and grad.dtype == torch.float32 and
                grad.is_contiguous() and grad.numel() == self.n_params):
            raise TypeError("grad must be a contiguous float32 CUDA tensor of n_params entries")
        _check(_lib.pdf_surrogate_adam(self.id, _P(grad.data_ptr()), float(lr), _stream(stream)))

    def grad(self, inp, target, stream=None):
        """(gradient tensor, loss tensor) for device float32 inp[B][2], target[B][16]."""
        g = torch.empty(self.n_params, dtype=torch.float32, device=inp.device)
        loss = torch.empty(1, dtype=torch.float32, device=inp.device)
        _check(_lib.pdf_surrogate_grad(self.id, _P(inp.data_ptr()), _P(target.data_ptr()), inp.shape[0],
                                       _P(g.data_ptr()), _P(loss.data_ptr()), _stream(stream)))
        return g, loss

    def params(self):
        a = np.empty(self.n_params, np.float32)
        _check(_lib.pdf_surrogate_params(self.id, _ptr(a), 0))
        return a

    def set_params(self, p):
        a = np.ascontiguousarray(p, np.float32)
        _check(_lib.pdf_surrogate_params(self.id, _ptr(a), 1))

    def xfxq2(self, x, q2, pids=None, out=None, n_cols=None, stream=None):
        """FP32 point-major [n][len(pids)] (pids=None: every stored column,
        then pass n_cols = number of stored columns, or out)."""
        _dev_f64(x, "x")
        _dev_f64(q2, "q2")
        arr, npid = _pid_arg(pids)
        if out is None:
            out = torch.empty((x.shape[0], npid if pids is not None else n_cols), dtype=torch.float32,
                              device=x.device)
        _check(_lib.pdf_surrogate_xfxq2(self.id, _ptr(arr) if arr is not None else None, npid, _P(x.data_ptr()),
                                        _P(q2.data_ptr()), x.shape[0], _P(out.data_ptr()), _stream(stream)))
        return out

    def save(self, path):
        _check(_lib.pdf_surrogate_save(self.id, str(path).encode()))

    def load(self, path):
        _check(_lib.pdf_surrogate_load(self.id, str(path).encode()))

    def destroy(self):
        if self.id >= 0:
            _check(_lib.pdf_surrogate_destroy(self.id))
            self.id = -1


def set_lds_policy(policy):
    _check(_lib.pdf_set_lds_policy(int(policy)))


def batch_tune_cache(path):
    """pdf_batch_tune_cache: keep autotune choices in the file at path (None stops appending)."""
    _check(_lib.pdf_batch_tune_cache(None if path is None else os.fsencode(path)))


TUNE_LDS_POLICY, TUNE_VECTOR_COLUMNS, TUNE_BLOCKS_PER_CU = 0, 1, 2


def set_tuning(knob, value):
    _check(_lib.pdf_set_tuning(int(knob), int(value)))


def get_tuning(knob):
    v = ctypes.c_int32(0)
    _check(_lib.pdf_get_tuning(int(knob), ctypes.byref(v)))
    return v.value


def shutdown():
    _check(_lib.pdf_shutdown())
