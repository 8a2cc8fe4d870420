"""Python binding of the C ABI (include/sdl.h) over torch device tensors.

torch provides device memory and the HIP stream; every step of the method runs
in libsdl.so.  Tensors are kept in the ABI's memory layout (column-major
matrices), so no data is reshaped on the way in:

    Y     (N, m2, m1)  signal k, pixel (i, j) at Y[k, j, i]
    D1    (n1, m1)     float64, atom i at D1[i, :]      (memory of the m1 x n1 column-major matrix)
    D2    (n2, m2)     float64
    supp  (N, s) int32, coef (N, s), res2 (N,)  (dtype of Y)

``Problem.from_math`` converts math-shaped inputs once.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _native

_DT = {torch.float64: _native.SDL_FP64, torch.float32: _native.SDL_FP32, torch.bfloat16: _native.SDL_BF16}
PRECISIONS = {"fp64": _native.SDL_FP64, "fp32": _native.SDL_FP32, "bf16": _native.SDL_BF16,
              "mixed_bf16": _native.SDL_MIXED_BF16}


class Problem:
    """One dictionary problem's device buffers, in ABI layout."""

    def __init__(self, Y: torch.Tensor, D1: torch.Tensor, D2: torch.Tensor, s: int,
                 supp: torch.Tensor | None = None, coef: torch.Tensor | None = None,
                 res2: torch.Tensor | None = None, with_res2: bool = True):
        if Y.dim() != 3 or D1.dim() != 2 or D2.dim() != 2:
            raise ValueError("Y must be (N, m2, m1), D1 (n1, m1), D2 (n2, m2)")
        self.N, self.m2, self.m1 = Y.shape
        self.n1, self.n2 = D1.shape[0], D2.shape[0]
        if D1.shape[1] != self.m1 or D2.shape[1] != self.m2:
            raise ValueError("dictionary row counts do not match the signal shape")
        if Y.dtype not in _DT:
            raise ValueError("Y must be float64, float32 or bfloat16")
        for t in (Y, D1, D2):
            if not t.is_contiguous():
                raise ValueError("tensors must be contiguous (ABI layout)")
        if D1.dtype != torch.float64 or D2.dtype != torch.float64:
            raise ValueError("dictionaries are FP64 master copies")
        self.s = int(s)
        dev = Y.device
        cdt = torch.float32 if Y.dtype == torch.bfloat16 else Y.dtype  # codes of BF16 signals are FP32
        self.Y, self.D1, self.D2 = Y, D1, D2
        self.supp = supp if supp is not None else torch.empty((self.N, self.s), dtype=torch.int32, device=dev)
        self.coef = coef if coef is not None else torch.empty((self.N, self.s), dtype=cdt, device=dev)
        self.res2 = res2 if res2 is not None else (
            torch.empty(self.N, dtype=cdt, device=dev) if with_res2 else None)

    @classmethod
    def from_math(cls, Y, D1, D2, s, dtype=torch.float32, device="cuda"):
        """Y (N, m1, m2), D1 (m1, n1), D2 (m2, n2) (numpy or torch) -> ABI-layout device buffers."""
        Y = torch.as_tensor(Y)
        D1 = torch.as_tensor(D1)
        D2 = torch.as_tensor(D2)
        Yc = Y.to(device=device, dtype=dtype).transpose(1, 2).contiguous()
        return cls(Yc, D1.to(device=device, dtype=torch.float64).t().contiguous(),
                   D2.to(device=device, dtype=torch.float64).t().contiguous(), s)

    @property
    def prec(self):
        return _DT[self.Y.dtype]

    def d1(self):
        """D1 in math shape (m1, n1), on the host."""
        return self.D1.t().cpu().numpy()

    def d2(self):
        return self.D2.t().cpu().numpy()

    def struct(self) -> _native.Problem:
        def p(t):
            return ctypes.c_void_p(t.data_ptr()) if t is not None else None
        return _native.Problem(self.m1, self.m2, self.n1, self.n2, self.s, 0, self.N, p(self.Y), p(self.D1),
                               p(self.D2), p(self.supp), p(self.coef), p(self.res2))


def _options(problems, stats=None, **kw):
    """Options for a call: the precision follows the signals' dtype; ``mixed=True`` asks for
    SDL_MIXED_BF16 (bfloat16 signals, correlations on the BF16 matrix cores)."""
    o = _native.default_options()
    precs = {pr.prec for pr in problems}
    if len(precs) > 1:
        raise ValueError("all problems of one call share a precision")
    o.prec = precs.pop() if precs else _native.SDL_FP64
    if kw.pop("mixed", False):
        if o.prec != _native.SDL_BF16:
            raise ValueError("mixed=True needs bfloat16 signals")
        o.prec = _native.SDL_MIXED_BF16
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    if stats is not None:
        o.stats = ctypes.pointer(stats)
    return o


def _array(problems):
    arr = (_native.Problem * max(1, len(problems)))()
    for i, pr in enumerate(problems):
        arr[i] = pr.struct()
    return arr


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def sparse_code(problems: Problem | Sequence[Problem], stream=None, stats=None, **opts):
    """2D-OMP of every signal of every problem (asynchronous on the stream)."""
    problems = [problems] if isinstance(problems, Problem) else list(problems)
    o = _options(problems, stats, **opts)
    arr = _array(problems)
    _native.check(_native.lib().sdl_sparse_code(arr, len(problems), ctypes.byref(o), _stream(stream)))
    return problems


def sparse_code_sums(problem: Problem, side: int, stream=None, stats=None, **opts) -> torch.Tensor:
    """2D-OMP of the problem's signals plus the reduced sums of one side's dictionary update
    (Algorithm 1 step 1 or 3): returns a float64 device tensor [A (na*na) | B (mr*na) | sum res2],
    A and B column-major (asynchronous on the stream)."""
    na, mr = (problem.n1, problem.m1) if side == 1 else (problem.n2, problem.m2)
    out = torch.empty(na * na + mr * na + 1, dtype=torch.float64, device=problem.Y.device)
    o = _options([problem], stats, **opts)
    arr = _array([problem])
    _native.check(_native.lib().sdl_sparse_code_sums(arr, side, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o),
                                                     _stream(stream)))
    return out


def split_sums(sums, side, problem: Problem):
    """(A, B, sum res2) in math shape from a sparse_code_sums result (host numpy)."""
    v = sums.cpu().numpy() if isinstance(sums, torch.Tensor) else sums
    na, mr = (problem.n1, problem.m1) if side == 1 else (problem.n2, problem.m2)
    A = v[:na * na].reshape(na, na).T
    B = v[na * na:na * na + mr * na].reshape(na, mr).T
    return A.copy(), B.copy(), float(v[-1])


def workspace_bytes(problems: Problem | Sequence[Problem], call: str = "learn", K: int = 0, **opts) -> int:
    """Workspace bytes a call needs when the caller supplies it (options ``workspace``)."""
    problems = [problems] if isinstance(problems, Problem) else list(problems)
    kinds = {"sparse_code": 0, "tmod_update": 1, "learn": 2, "sparse_code_sums": 3}
    o = _options(problems, None, **opts)
    n = ctypes.c_size_t()
    _native.check(_native.lib().sdl_workspace_bytes(_array(problems), len(problems), kinds[call], K,
                                                    ctypes.byref(o), ctypes.byref(n)))
    return n.value


def image_to_patches(image: torch.Tensor, m1: int, m2: int, stream=None) -> torch.Tensor:
    """All overlapping m1 x m2 patches (stride 1) of a row-major (H, W) float32/float64 device image,
    as signals in ABI layout: (N, m2, m1) with N = (H - m1 + 1)(W - m2 + 1)."""
    if image.dim() != 2 or not image.is_contiguous():
        raise ValueError("image must be a contiguous (H, W) tensor")
    H, W = image.shape
    prec = _DT[image.dtype]
    out = torch.empty(((H - m1 + 1) * (W - m2 + 1), m2, m1), dtype=image.dtype, device=image.device)
    _native.check(_native.lib().sdl_image_to_patches(ctypes.c_void_p(image.data_ptr()), H, W, m1, m2, prec,
                                                     ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def patches_to_image(problem: Problem, H: int, W: int, stream=None, **opts) -> torch.Tensor:
    """The (H, W) image rebuilt from the problem's codes of those patches (plain average of the
    overlapping estimates)."""
    out = torch.empty((H, W), dtype=problem.coef.dtype, device=problem.coef.device)
    o = _options([problem], None, **opts)
    _native.check(_native.lib().sdl_patches_to_image(_array([problem]), H, W, ctypes.byref(o),
                                                     ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def denoise(noisy: torch.Tensor, D1: torch.Tensor, D2: torch.Tensor, sigma: float, s_cap: int | None = None,
            c_eps: float = 1.15, stream=None, stats=None, **opts):
    """The denoising experiment of Sec. IV on one image: every overlapping patch of ``noisy`` (H, W) is
    coded by the error-driven 2D-OMP with eps = c_eps sigma sqrt(m1 m2) and at most s_cap atoms (default
    m1 m2 / 2), and the image is rebuilt from the codes.  D1 (n1, m1), D2 (n2, m2) are FP64 device
    dictionaries in ABI layout.  Returns (denoised image, the coded problem)."""
    n1, m1 = D1.shape
    n2, m2 = D2.shape
    P = image_to_patches(noisy, m1, m2, stream=stream)
    s = s_cap if s_cap is not None else m1 * m2 // 2
    pr = Problem(P, D1, D2, s)
    err2 = (c_eps * sigma) ** 2 * m1 * m2
    sparse_code(pr, stream=stream, stats=stats, err2=err2, **opts)
    H, W = noisy.shape
    return patches_to_image(pr, H, W, stream=stream), pr


class TensorProblem:
    """n-dimensional signals (Remark 3) in ABI layout: Y (N, m_n, ..., m_1) contiguous, i.e. each
    signal stored first index fastest; dictionaries D_d as FP64 (n_d, m_d) tensors (column-major
    m_d x n_d)."""

    def __init__(self, Y: torch.Tensor, Ds, s: int, with_res2: bool = True):
        nm = len(Ds)
        if not 2 <= nm <= _native.TENSOR_MAX_MODES or Y.dim() != nm + 1:
            raise ValueError("Y must be (N, m_n, ..., m_1) with 2..4 modes, one dictionary per mode")
        if Y.dtype not in (torch.float64, torch.float32) or not Y.is_contiguous():
            raise ValueError("Y must be a contiguous float64 or float32 tensor")
        self.m = [int(x) for x in reversed(Y.shape[1:])]
        self.n = [int(D.shape[0]) for D in Ds]
        for d, D in enumerate(Ds):
            if D.dtype != torch.float64 or not D.is_contiguous() or D.shape[1] != self.m[d]:
                raise ValueError("dictionary %d must be a contiguous float64 (n_d, m_d) tensor" % (d + 1))
        self.N, self.s, self.Y, self.Ds = int(Y.shape[0]), int(s), Y, list(Ds)
        dev = Y.device
        self.supp = torch.empty((self.N, self.s), dtype=torch.int32, device=dev)
        self.coef = torch.empty((self.N, self.s), dtype=Y.dtype, device=dev)
        self.res2 = torch.empty(self.N, dtype=Y.dtype, device=dev) if with_res2 else None

    @classmethod
    def from_math(cls, Y, Ds, s, dtype=torch.float64, device="cuda"):
        """Y (N, m_1, ..., m_n), D_d (m_d, n_d) (numpy or torch) -> ABI-layout device buffers."""
        Y = torch.as_tensor(Y)
        nm = Y.dim() - 1
        Yc = Y.to(device=device, dtype=dtype).permute(0, *range(nm, 0, -1)).contiguous()
        return cls(Yc, [torch.as_tensor(D).to(device=device, dtype=torch.float64).t().contiguous() for D in Ds], s)

    def dicts(self):
        """The dictionaries in math shape (m_d, n_d), on the host."""
        return [D.t().cpu().numpy() for D in self.Ds]

    def struct(self) -> _native.TensorProblem:
        t = _native.TensorProblem()
        t.nmodes, t.s, t.N = len(self.Ds), self.s, self.N
        for d in range(len(self.Ds)):
            t.m[d], t.n[d] = self.m[d], self.n[d]
            t.D[d] = self.Ds[d].data_ptr()
        t.Y = self.Y.data_ptr()
        t.supp, t.coef = self.supp.data_ptr(), self.coef.data_ptr()
        t.res2 = self.res2.data_ptr() if self.res2 is not None else None
        return t


def _tensor_options(problem: TensorProblem, stats=None, **kw):
    o = _native.default_options()
    o.prec = _DT[problem.Y.dtype]
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    if stats is not None:
        o.stats = ctypes.pointer(stats)
    return o


def tensor_sparse_code(problem: TensorProblem, stream=None, stats=None, **opts):
    o = _tensor_options(problem, stats, **opts)
    t = problem.struct()
    _native.check(_native.lib().sdl_tensor_sparse_code(ctypes.byref(t), ctypes.byref(o), _stream(stream)))
    return problem


def tensor_update(problem: TensorProblem, mode: int, stream=None, stats=None, **opts):
    o = _tensor_options(problem, stats, **opts)
    t = problem.struct()
    _native.check(_native.lib().sdl_tensor_update(ctypes.byref(t), mode, ctypes.byref(o), _stream(stream)))
    return problem


def tensor_learn(problem: TensorProblem, K: int, stream=None, stats=None, **opts) -> np.ndarray:
    """Algorithm 1 with one sweep per mode; returns the RMSE trace (K + 1 values)."""
    o = _tensor_options(problem, stats, **opts)
    t = problem.struct()
    trace = np.zeros(K + 1)
    _native.check(_native.lib().sdl_tensor_learn(ctypes.byref(t), K, trace.ctypes.data_as(ctypes.c_void_p),
                                                 ctypes.byref(o), _stream(stream)))
    return trace


def mixed_supported(m1, m2, n1, n2, s) -> bool:
    return bool(_native.lib().sdl_mixed_supported(m1, m2, n1, n2, s))


def tmod_update(problems: Problem | Sequence[Problem], sides: int = 3, stream=None, stats=None, **opts):
    """Dictionary update(s) from the current codes; rescales coef in place.  Synchronises."""
    problems = [problems] if isinstance(problems, Problem) else list(problems)
    o = _options(problems, stats, **opts)
    arr = _array(problems)
    _native.check(_native.lib().sdl_tmod_update(arr, len(problems), sides, ctypes.byref(o), _stream(stream)))
    return problems


def learn(problems: Problem | Sequence[Problem], K: int, stream=None, stats=None, proposer=None, tau=0.0, **opts):
    """Algorithm 1 for K iterations plus a final sparse coding.  Returns the RMSE trace (nprob, K+1).
    With ``proposer`` every sparse coding uses the learned proposal with 2D-OMP fallback."""
    import numpy as np
    problems = [problems] if isinstance(problems, Problem) else list(problems)
    o = _options(problems, stats, **opts)
    if proposer is not None:
        o.proposer = proposer.handle
        o.tau = tau
    arr = _array(problems)
    trace = np.zeros((max(1, len(problems)), K + 1), dtype=np.float64)
    st = _native.lib().sdl_learn(arr, len(problems), K, trace.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o),
                                 _stream(stream))
    _native.check(st)
    return trace[:len(problems)]


def autotune(problems: Problem | Sequence[Problem], reps: int = 5, stream=None, **opts):
    """Time the register-resident kernel variants on these problems and keep the fastest."""
    problems = [problems] if isinstance(problems, Problem) else list(problems)
    o = _options(problems, None, **opts)
    arr = _array(problems)
    _native.check(_native.lib().sdl_autotune(arr, len(problems), reps, ctypes.byref(o), _stream(stream)))


def tuned_config(m1, m2, n1, n2, s):
    """(lanes_row, lanes_col, waves_per_simd, matrix_core, tuned_ms) for an FP32 shape, or None."""
    a, b, c, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_double()
    st = _native.lib().sdl_tuned_config(m1, m2, n1, n2, s, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                        ctypes.byref(d), ctypes.byref(ms))
    if st != 0:
        return None
    return a.value, b.value, c.value, d.value, ms.value


def kernel_variants(m1, m2, n1, n2, s):
    """[(lanes_row, lanes_col, waves_per_simd, matrix_core), ...] compiled for an FP32 shape."""
    buf = (ctypes.c_int32 * 256)()
    n = _native.lib().sdl_kernel_variants(m1, m2, n1, n2, s, buf, 64)
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(min(n, 64))]


def set_kernel_variant(m1, m2, n1, n2, s, variant):
    _native.check(_native.lib().sdl_set_kernel_variant(m1, m2, n1, n2, s, *variant))


class Proposer:
    """Learned support proposal network (see sdl_proposer_* in include/sdl.h).

    Weights live on the device; ``params``/``set_params`` move the flat FP32 master
    vector [W1 (hidden x m1m2), b1, W2, b2, W3 (n1n2 x hidden), b3]."""

    def __init__(self, m1, m2, n1, n2, hidden=512, fp32_check=False, seed=7):
        self._h = ctypes.c_void_p()
        _native.check(_native.lib().sdl_proposer_create(m1, m2, n1, n2, hidden, int(bool(fp32_check)), seed,
                                                        ctypes.byref(self._h)))
        self.m1, self.m2, self.n1, self.n2, self.hidden = m1, m2, n1, n2, hidden

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and h.value:
                _native.lib().sdl_proposer_destroy(h)
        except Exception:  # interpreter shutdown: the library may already be gone
            pass
        self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def num_params(self):
        return int(_native.lib().sdl_proposer_num_params(self._h))

    def params(self):
        import numpy as np
        out = np.empty(self.num_params, np.float32)
        _native.check(_native.lib().sdl_proposer_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.num_params
        _native.check(_native.lib().sdl_proposer_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)))

    def gradient(self, Y: torch.Tensor, supp: torch.Tensor, s: int, stream=None):
        """(mean BCE loss, flat FP32 gradient) on the B signals of Y (ABI layout, B % 64 == 0)."""
        import numpy as np
        g = np.empty(self.num_params, np.float32)
        loss = ctypes.c_double()
        _native.check(_native.lib().sdl_proposer_gradient(
            self._h, ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(supp.data_ptr()), s, Y.shape[0],
            g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss), _stream(stream)))
        return loss.value, g

    def train(self, Y: torch.Tensor, supp: torch.Tensor, s: int, epochs=5, batch=1024, lr=1e-3, seed=8, stream=None):
        import numpy as np
        tr = np.zeros(max(1, epochs))
        _native.check(_native.lib().sdl_proposer_train(
            self._h, ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(supp.data_ptr()), s, Y.shape[0], epochs, batch,
            lr, seed, tr.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return tr[:epochs]

    def logits(self, Y: torch.Tensor, stream=None):
        out = torch.empty((Y.shape[0], self.n1 * self.n2), dtype=torch.float32, device=Y.device)
        _native.check(_native.lib().sdl_proposer_logits(self._h, ctypes.c_void_p(Y.data_ptr()), Y.shape[0],
                                                        ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def calibrate(self, problem: Problem, violation=0.01, fallback_margin=1.01, stream=None):
        tau = ctypes.c_double()
        arr = _array([problem])
        o = _native.default_options()
        o.prec = _native.SDL_FP32
        o.fallback_margin = fallback_margin
        _native.check(_native.lib().sdl_proposer_calibrate(self._h, arr, violation, ctypes.byref(o),
                                                           ctypes.byref(tau), _stream(stream)))
        return tau.value

    def save(self, path):
        _native.check(_native.lib().sdl_proposer_save(self._h, str(path).encode()))

    @classmethod
    def load(cls, path):
        import struct
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p()
        _native.check(_native.lib().sdl_proposer_load(str(path).encode(), ctypes.byref(self._h)))
        with open(path, "rb") as f:  # the header's sizes (the library has validated the file)
            self.m1, self.m2, self.n1, self.n2, self.hidden, _ = struct.unpack("<6i", f.read(32)[8:32])
        return self


def learned_sparse_code(proposer: Proposer, problems, tau: float, accept: torch.Tensor | None = None, stream=None,
                        stats=None, **opts):
    """Proposal + least squares, 2D-OMP for the rejected signals (FP32 problems)."""
    problems = [problems] if isinstance(problems, Problem) else list(problems)
    o = _options(problems, stats, **opts)
    o.tau = tau
    arr = _array(problems)
    acc = ctypes.c_void_p(accept.data_ptr()) if accept is not None else None
    _native.check(_native.lib().sdl_learned_sparse_code(proposer.handle, arr, len(problems), acc, ctypes.byref(o),
                                                        _stream(stream)))
    return problems


def new_stats() -> _native.Stats:
    return _native.Stats()


PROBE_KINDS = {"fp32_fma": 0, "fp32_mfma_16x16x4": 1, "fp32_mfma_4x4x1": 2, "fp64_fma": 3,
               "bf16_mfma_4x4x4": 4, "bf16_mfma_16x16x16": 5, "bf16_mfma_16x16x32": 6}


def probe_hbm_copy(nbytes: int = 1 << 30, reps: int = 5, stream=None) -> float:
    """Best device copy rate, read + write bytes, in GB/s (buffers allocated here)."""
    src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    gbs = ctypes.c_double()
    _native.check(_native.lib().sdl_probe_hbm_copy(dst.data_ptr(), src.data_ptr(), nbytes, reps, ctypes.byref(gbs),
                                                   _stream(stream)))
    return gbs.value


def probe_peak(kind: str, reps: int = 5, stream=None) -> float:
    """Achievable arithmetic peak in TFLOP/s; kind in PROBE_KINDS."""
    sink = torch.zeros(2, dtype=torch.float64, device="cuda")
    tf = ctypes.c_double()
    _native.check(_native.lib().sdl_probe_peak(PROBE_KINDS[kind], sink.data_ptr(), reps, ctypes.byref(tf),
                                               _stream(stream)))
    return tf.value
