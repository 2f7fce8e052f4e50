"""MI355X (gfx950) dense Pauli decomposition.

Python binding of libpauli (include/pauli.h): every computation runs in the
library's HIP kernels; this module only marshals torch tensors (device memory
and the current stream) into the C ABI.  It raises if the library is not
built or no GPU is visible -- there is no CPU fallback.

    c = decompose(G)            # G: complex [..., 2^N, 2^N] on cuda -> [..., 4^N]
    G = reconstruct(c)          # sum_n c_n P_n
    g = decompose_backward(gc)  # 2^-N sum_n gc_n P_n  (adjoint of decompose)
    cs = decompose_batched([G0, G1, ...])   # uneven N, one persistent launch
    PauliDecompose.apply(G)     # differentiable

Coefficient n takes operator t (0=I, 1=X, 2=Y, 3=Z) from bits (2t+1, 2t);
qubit t is the t-th Kronecker factor from the right (T. Jones 2024, section 2).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpauli.so")

ALGOS = {"fp64_gray": 0, "fp32": 1, "split_bf16": 2, "fwht": 3, "split_fp16": 4, "fwht_f32": 5, "split_i8": 6}
_DT = {torch.complex64: 0, torch.complex128: 1}
_TORCH_DT = {0: torch.complex64, 1: torch.complex128}
_STATUS = {0: "OK", 1: "EINVAL", 2: "EUNSUPPORTED", 3: "EHIP", 4: "ENOMEM"}


class PauliError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("pauli status %s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("in_dtype", ctypes.c_int), ("out_dtype", ctypes.c_int),
                ("tile", ctypes.c_int), ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


_lib = None
_lock = threading.Lock()

EXPORTS = ["pauli_opts_default", "pauli_decompose", "pauli_reconstruct", "pauli_decompose_backward",
           "pauli_decompose_batched", "pauli_batched_workspace_bytes", "pauli_workspace_bytes",
           "pauli_batched_tile_count", "pauli_batched_tile_valid", "pauli_autotune_batched",
           "pauli_batched_tile_selected", "pauli_autotune", "pauli_tile_count", "pauli_tile_valid",
           "pauli_tile_selected", "pauli_pack", "pauli_contract", "pauli_coeffs_at", "pauli_coeffs_at_backward",
           "pauli_decompose_hermitian", "pauli_tile_valid_hermitian",
           "pauli_coeffs_at_workspace_bytes", "pauli_last_error", "pauli_version",
           "pauli_decompose_noalloc", "pauli_noalloc_scratch_bytes", "pauli_tile_selected_hermitian"]


def load_library(path: str = LIB_PATH):
    """Load libpauli.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError("libpauli.so is not built (python -m paper_2401_16378_amd.build)")
        lib = ctypes.CDLL(path)
        vp, ci, op = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Opts)
        lib.pauli_opts_default.argtypes = [op]
        lib.pauli_opts_default.restype = None
        for name in ("pauli_decompose", "pauli_reconstruct", "pauli_decompose_backward",
                     "pauli_decompose_hermitian", "pauli_decompose_noalloc"):
            getattr(lib, name).argtypes = [vp, ci, ci, vp, op]
            getattr(lib, name).restype = ci
        lib.pauli_decompose_batched.argtypes = [ci, ctypes.POINTER(vp), ctypes.POINTER(ci),
                                                ctypes.POINTER(vp), op]
        lib.pauli_decompose_batched.restype = ci
        ip = ctypes.POINTER(ci)
        lib.pauli_batched_workspace_bytes.argtypes = [ci, ip, ci]
        lib.pauli_batched_workspace_bytes.restype = ctypes.c_size_t
        lib.pauli_autotune_batched.argtypes = [ci, ctypes.POINTER(vp), ip, ctypes.POINTER(vp), op]
        lib.pauli_autotune_batched.restype = ci
        lib.pauli_batched_tile_count.argtypes = []
        lib.pauli_batched_tile_count.restype = ci
        lib.pauli_batched_tile_valid.argtypes = [ci, ci]
        lib.pauli_batched_tile_valid.restype = ci
        lib.pauli_batched_tile_selected.argtypes = [ci, ip, ci]
        lib.pauli_batched_tile_selected.restype = ci
        lib.pauli_workspace_bytes.argtypes = [ci, ci, ci]
        lib.pauli_workspace_bytes.restype = ctypes.c_size_t
        lib.pauli_autotune.argtypes = [ci, ci, op]
        lib.pauli_autotune.restype = ci
        lib.pauli_tile_count.argtypes = [ci]
        lib.pauli_tile_count.restype = ci
        lib.pauli_tile_valid.argtypes = [ci, ci, ci]
        lib.pauli_tile_valid.restype = ci
        lib.pauli_tile_valid_hermitian.argtypes = [ci, ci, ci]
        lib.pauli_tile_valid_hermitian.restype = ci
        lib.pauli_tile_selected.argtypes = [ci, ci]
        lib.pauli_tile_selected.restype = ci
        lib.pauli_tile_selected_hermitian.argtypes = [ci, ci]
        lib.pauli_tile_selected_hermitian.restype = ci
        lib.pauli_pack.argtypes = [vp, ci, ci, ci, op]
        lib.pauli_pack.restype = ci
        lib.pauli_contract.argtypes = [ci, ci, ci, vp, op]
        lib.pauli_contract.restype = ci
        lib.pauli_coeffs_at.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_uint), ci, vp, op]
        lib.pauli_coeffs_at.restype = ci
        lib.pauli_coeffs_at_backward.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_uint), ci, vp, op]
        lib.pauli_coeffs_at_backward.restype = ci
        lib.pauli_coeffs_at_workspace_bytes.argtypes = [ci, ci]
        lib.pauli_coeffs_at_workspace_bytes.restype = ctypes.c_size_t
        lib.pauli_last_error.argtypes = []
        lib.pauli_last_error.restype = ctypes.c_char_p
        lib.pauli_noalloc_scratch_bytes.argtypes = []
        lib.pauli_noalloc_scratch_bytes.restype = ctypes.c_size_t
        lib.pauli_version.argtypes = []
        lib.pauli_version.restype = ci
        _lib = lib
        return lib


def last_error() -> str:
    return load_library().pauli_last_error().decode()


def _check(status: int):
    if status != 0:
        raise PauliError(status, last_error())


def _opts(algo: str, in_dt: int, out_dt: int, tile: int = 0, stream=None, workspace=None) -> _Opts:
    o = _Opts()
    o.algo = ALGOS[algo]
    o.in_dtype = in_dt
    o.out_dtype = out_dt
    o.tile = tile
    o.stream = stream
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


_scratch = {}   # (device, stream) -> scratch buffer, insertion order = recency
_SCRATCH_KEEP = 8


def workspace(algo: str, N: int, batch: int, device) -> torch.Tensor:
    """A cached device scratch buffer large enough for (algo, N, batch) on
    torch's current stream of `device`, or None when the algorithm needs
    none.  Each stream has its own buffer, reused by the calls enqueued on it
    (which run in order), so work on different streams never shares one."""
    need = load_library().pauli_workspace_bytes(ALGOS[algo], N, batch)
    if need == 0:
        return None
    dev = torch.device(device)
    key = (dev, torch.cuda.current_stream(dev).cuda_stream)
    ws = _scratch.pop(key, None)
    if ws is None or ws.numel() < need:
        while len(_scratch) >= _SCRATCH_KEEP:   # least recently used first (freed in stream order)
            _scratch.pop(next(iter(_scratch)))
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    _scratch[key] = ws                           # most recently used last
    return ws


def release_workspace(device=None) -> None:
    """Drop the cached scratch buffers of `device` (all devices if None)."""
    if device is None:
        _scratch.clear()
    else:
        dev = torch.device(device)
        for key in [k for k in _scratch if k[0] == dev]:
            del _scratch[key]


def _on(dev):
    """The library launches on the current HIP device: make `dev` current for
    the duration of a call."""
    return torch.cuda.device(dev)


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _qubits_of_matrix(G: torch.Tensor) -> int:
    D = G.shape[-1]
    if G.dim() < 2 or G.shape[-2] != D or D & (D - 1):
        raise ValueError("expected [..., 2^N, 2^N], got %s" % (tuple(G.shape),))
    return D.bit_length() - 1


def _qubits_of_coeffs(c: torch.Tensor) -> int:
    L = c.shape[-1]
    N = (L.bit_length() - 1) // 2
    if c.dim() < 1 or L != 1 << (2 * N):
        raise ValueError("expected [..., 4^N], got %s" % (tuple(c.shape),))
    return N


def _prep(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("tensor must be on a GPU device")
    if t.dtype not in _DT:
        raise TypeError("tensor must be complex64 or complex128, got %s" % t.dtype)
    t = t.contiguous()
    # The C ABI takes 16-byte aligned pointers only (the matrix-core paths
    # read complex64 input in 16-byte pairs); a view starting at an odd
    # complex64 element is copied into a fresh (aligned) allocation.
    return t if t.data_ptr() % 16 == 0 else t.clone()


def decompose(G: torch.Tensor, algo: str = "split_bf16", out_dtype=None, tile: int = 0) -> torch.Tensor:
    """c[..., n] = 2^-N Tr(P_n G[...]) for complex G of shape [..., 2^N, 2^N]."""
    G = _prep(G)
    N = _qubits_of_matrix(G)
    out_dtype = out_dtype or G.dtype
    batch = G.numel() // (1 << (2 * N))
    out = torch.empty(G.shape[:-2] + (1 << (2 * N),), dtype=out_dtype, device=G.device)
    o = _opts(algo, _DT[G.dtype], _DT[out_dtype], tile, _stream(G), workspace(algo, N, batch, G.device))
    with _on(G.device):
        _check(load_library().pauli_decompose(G.data_ptr(), N, batch, out.data_ptr(), ctypes.byref(o)))
    return out


def decompose_noalloc(G: torch.Tensor, algo: str = "split_bf16", out_dtype=None, tile: int = 0) -> torch.Tensor:
    """decompose() through pauli_decompose_noalloc: the library's fixed
    per-GPU scratch instead of a workspace (only the output is allocated
    here, by torch)."""
    G = _prep(G)
    N = _qubits_of_matrix(G)
    out_dtype = out_dtype or G.dtype
    batch = G.numel() // (1 << (2 * N))
    out = torch.empty(G.shape[:-2] + (1 << (2 * N),), dtype=out_dtype, device=G.device)
    o = _opts(algo, _DT[G.dtype], _DT[out_dtype], tile, _stream(G))
    with _on(G.device):
        _check(load_library().pauli_decompose_noalloc(G.data_ptr(), N, batch, out.data_ptr(), ctypes.byref(o)))
    return out


def decompose_hermitian(G: torch.Tensor, algo: str = "split_bf16", out_dtype=None, tile: int = 0) -> torch.Tensor:
    """decompose() for Hermitian G: half the matrix-core work for most flip
    masks, coefficients with imaginary part exactly zero.  G being Hermitian
    is the caller's promise (not checked; otherwise the result is
    unspecified).  Not differentiable: use PauliDecompose for gradients."""
    if G.requires_grad:
        raise ValueError("decompose_hermitian has no gradient; use PauliDecompose")
    G = _prep(G)
    N = _qubits_of_matrix(G)
    out_dtype = out_dtype or G.dtype
    batch = G.numel() // (1 << (2 * N))
    out = torch.empty(G.shape[:-2] + (1 << (2 * N),), dtype=out_dtype, device=G.device)
    o = _opts(algo, _DT[G.dtype], _DT[out_dtype], tile, _stream(G), workspace(algo, N, batch, G.device))
    with _on(G.device):
        _check(load_library().pauli_decompose_hermitian(G.data_ptr(), N, batch, out.data_ptr(), ctypes.byref(o)))
    return out


def reconstruct(c: torch.Tensor, algo: str = "split_bf16", out_dtype=None, tile: int = 0) -> torch.Tensor:
    """G = sum_n c_n P_n for c of shape [..., 4^N]."""
    c = _prep(c)
    N = _qubits_of_coeffs(c)
    out_dtype = out_dtype or c.dtype
    D = 1 << N
    batch = c.numel() // (D * D)
    G = torch.empty(c.shape[:-1] + (D, D), dtype=out_dtype, device=c.device)
    o = _opts(algo, _DT[c.dtype], _DT[out_dtype], tile, _stream(c), workspace(algo, N, batch, c.device))
    with _on(c.device):
        _check(load_library().pauli_reconstruct(c.data_ptr(), N, batch, G.data_ptr(), ctypes.byref(o)))
    return G


def decompose_backward(grad_c: torch.Tensor, algo: str = "split_bf16", out_dtype=None,
                       tile: int = 0) -> torch.Tensor:
    """Adjoint of decompose: 2^-N sum_n grad_c[n] P_n."""
    g = _prep(grad_c)
    N = _qubits_of_coeffs(g)
    out_dtype = out_dtype or g.dtype
    D = 1 << N
    batch = g.numel() // (D * D)
    G = torch.empty(g.shape[:-1] + (D, D), dtype=out_dtype, device=g.device)
    o = _opts(algo, _DT[g.dtype], _DT[out_dtype], tile, _stream(g), workspace(algo, N, batch, g.device))
    with _on(g.device):
        _check(load_library().pauli_decompose_backward(g.data_ptr(), N, batch, G.data_ptr(), ctypes.byref(o)))
    return G


_batch_ws = {}          # (device, stream, algo, N list) -> workspace, insertion order = recency
_BATCH_WS_KEEP = 16


def coeffs_at(G: torch.Tensor, strings, out_dtype=None, workspace_tensor=None) -> torch.Tensor:
    """c_k = 2^-N Tr(P_{strings[k]} G) for one complex matrix G [2^N, 2^N] and a
    host list of string indices, O(2^N) each, summed in binary64."""
    import numpy as np
    G = _prep(G)
    N = _qubits_of_matrix(G)
    if G.dim() != 2:
        raise ValueError("coeffs_at takes one matrix, got shape %s" % (tuple(G.shape),))
    ns = np.ascontiguousarray(np.asarray(strings, dtype=np.uint64).reshape(-1))
    if ns.size and int(ns.max()) >= 1 << (2 * N):
        raise ValueError("string index %d is not below 4^%d" % (int(ns.max()), N))
    ns = ns.astype(np.uint32)
    out_dtype = out_dtype or G.dtype
    out = torch.empty(ns.shape[0], dtype=out_dtype, device=G.device)
    if ns.shape[0] == 0:
        return out
    o = _opts("fp64_gray", _DT[G.dtype], _DT[out_dtype], 0, _stream(G))
    if workspace_tensor is not None:
        o.workspace = workspace_tensor.data_ptr()
        o.workspace_bytes = workspace_tensor.numel() * workspace_tensor.element_size()
    with _on(G.device):
        _check(load_library().pauli_coeffs_at(G.data_ptr(), N, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_uint)),
                                              ns.shape[0], out.data_ptr(), ctypes.byref(o)))
    return out


def coeffs_at_backward(grad_c: torch.Tensor, N: int, strings, out_dtype=None, workspace_tensor=None) -> torch.Tensor:
    """Adjoint of coeffs_at: 2^-N sum_k grad_c[k] P_{strings[k]} as a dense
    [2^N, 2^N] tensor (binary64 sums)."""
    import numpy as np
    g = _prep(grad_c)
    ns = np.ascontiguousarray(np.asarray(strings, dtype=np.uint64).reshape(-1))
    if g.dim() != 1 or g.shape[0] != ns.shape[0]:
        raise ValueError("grad_c must be 1-D with one value per string")
    if ns.size and int(ns.max()) >= 1 << (2 * N):
        raise ValueError("string index %d is not below 4^%d" % (int(ns.max()), N))
    ns = ns.astype(np.uint32)
    out_dtype = out_dtype or g.dtype
    out = torch.empty((1 << N, 1 << N), dtype=out_dtype, device=g.device)
    if ns.shape[0] == 0:
        return out.zero_()
    o = _opts("fp64_gray", _DT[g.dtype], _DT[out_dtype], 0, _stream(g))
    if workspace_tensor is not None:
        o.workspace = workspace_tensor.data_ptr()
        o.workspace_bytes = workspace_tensor.numel() * workspace_tensor.element_size()
    with _on(g.device):
        _check(load_library().pauli_coeffs_at_backward(g.data_ptr(), N, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_uint)),
                                                       ns.shape[0], out.data_ptr(), ctypes.byref(o)))
    return out


def _batch_args(mats, algo, outs):
    mats = [_prep(m) for m in mats]
    for m in mats:
        if m.dtype != torch.complex64:
            raise TypeError("decompose_batched takes complex64 matrices")
    count = len(mats)
    dev = mats[0].device
    Ns = [_qubits_of_matrix(m) for m in mats]
    for m in mats:
        if m.device != dev:
            raise ValueError("all matrices must be on one device, got %s and %s" % (dev, m.device))
        if m.dim() != 2:
            raise ValueError("decompose_batched takes single matrices, got shape %s" % (tuple(m.shape),))
    if outs is None:
        outs = [torch.empty(1 << (2 * n), dtype=torch.complex64, device=dev) for n in Ns]
    else:
        outs = list(outs)
        if len(outs) != count:
            raise ValueError("%d outputs for %d matrices" % (len(outs), count))
        for o, n in zip(outs, Ns):   # the kernels write 4^N values through each pointer
            if o.device != dev or o.dtype != torch.complex64 or not o.is_contiguous() or o.numel() != 1 << (2 * n):
                raise ValueError("each output must be a contiguous complex64 tensor of 4^N values on %s" % dev)
    lib = load_library()
    Na = (ctypes.c_int * count)(*Ns)
    need = lib.pauli_batched_workspace_bytes(count, Na, ALGOS[algo])
    key = (dev, torch.cuda.current_stream(dev).cuda_stream, algo, tuple(Ns))   # per stream: no sharing
    ws = _batch_ws.pop(key, None)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        while len(_batch_ws) >= _BATCH_WS_KEEP:   # least recently used first (freed in stream order)
            _batch_ws.pop(next(iter(_batch_ws)))
    _batch_ws[key] = ws                           # most recently used last
    Gp = (ctypes.c_void_p * count)(*[m.data_ptr() for m in mats])
    Op = (ctypes.c_void_p * count)(*[o.data_ptr() for o in outs])
    return mats, outs, count, Na, Gp, Op, ws


def decompose_batched(mats, algo: str = "split_bf16", outs=None, tile: int = 0):
    """Decompose complex64 matrices of uneven size: one batched pack launch and
    one persistent contraction launch, replayed from a cached HIP graph.
    Returns a list of coefficient tensors (or fills `outs`).  The workspace is
    cached per N list, so repeated calls with the same sizes replay the graph."""
    if len(mats) == 0:
        return []
    mats, outs, count, Na, Gp, Op, ws = _batch_args(mats, algo, outs)
    o = _opts(algo, 0, 0, tile, _stream(mats[0]), ws)
    with _on(mats[0].device):
        _check(load_library().pauli_decompose_batched(count, Gp, Na, Op, ctypes.byref(o)))
    return outs


class BatchPlan:
    """decompose_batched for a fixed list of matrices and outputs, marshalled
    once: run() is one library call (a descriptor copy and a HIP graph
    replay), for loops that decompose the same buffers again and again.
    The tensors must stay alive and keep their storage while the plan is
    used; run() enqueues on torch's current stream of their device."""

    def __init__(self, mats, algo: str = "split_bf16", outs=None, tile: int = 0):
        if len(mats) == 0:
            raise ValueError("BatchPlan needs at least one matrix")
        (self.mats, self.outs, self.count, self._Na, self._Gp, self._Op,
         self._ws) = _batch_args(mats, algo, outs)
        self._dev = self.mats[0].device
        self._o = _opts(algo, 0, 0, tile, _stream(self.mats[0]), self._ws)
        self._lib = load_library()

    def run(self):
        self._o.stream = ctypes.c_void_p(torch.cuda.current_stream(self._dev).cuda_stream)
        with _on(self._dev):
            _check(self._lib.pauli_decompose_batched(self.count, self._Gp, self._Na, self._Op, ctypes.byref(self._o)))
        return self.outs


def autotune_batched(mats, algo: str = "split_bf16", outs=None) -> int:
    """Time every persistent tile shape on this batch and keep the fastest for
    its N list; returns the chosen tile (outputs hold the decomposition)."""
    mats, outs, count, Na, Gp, Op, ws = _batch_args(mats, algo, outs)
    o = _opts(algo, 0, 0, 0, _stream(mats[0]), ws)
    lib = load_library()
    with _on(mats[0].device):
        _check(lib.pauli_autotune_batched(count, Gp, Na, Op, ctypes.byref(o)))
    return lib.pauli_batched_tile_selected(count, Na, ALGOS[algo])


def autotune(n_min: int, n_max: int, algo: str = "split_bf16", device=None) -> dict:
    """Time every tile id for n_min..n_max and keep the fastest (blocking)."""
    dev = torch.device(device or "cuda")
    o = _opts(algo, 0, 0, 0, ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    lib = load_library()
    with _on(dev):
        _check(lib.pauli_autotune(n_min, n_max, ctypes.byref(o)))
    return {n: lib.pauli_tile_selected(ALGOS[algo], n) for n in range(n_min, n_max + 1)}


def tile_count(algo: str = "split_bf16") -> int:
    return load_library().pauli_tile_count(ALGOS[algo])


def tile_valid(tile: int, N: int, algo: str = "split_bf16") -> bool:
    return bool(load_library().pauli_tile_valid(ALGOS[algo], tile, N))


def tile_valid_hermitian(tile: int, N: int, algo: str = "split_bf16") -> bool:
    return bool(load_library().pauli_tile_valid_hermitian(ALGOS[algo], tile, N))


def batched_tile_valid(tile: int, algo: str = "split_bf16") -> bool:
    return bool(load_library().pauli_batched_tile_valid(ALGOS[algo], tile))


def tile_selected(N: int, algo: str = "split_bf16") -> int:
    return load_library().pauli_tile_selected(ALGOS[algo], N)


def tile_selected_hermitian(N: int, algo: str = "split_bf16") -> int:
    return load_library().pauli_tile_selected_hermitian(ALGOS[algo], N)


from .autograd import PauliCoeffsAt, PauliDecompose  # noqa: E402

__all__ = ["BatchPlan", "decompose", "decompose_hermitian", "tile_valid_hermitian", "reconstruct", "decompose_backward", "decompose_batched", "coeffs_at",
           "coeffs_at_backward", "PauliCoeffsAt", "autotune",
           "autotune_batched", "workspace", "release_workspace", "tile_valid", "batched_tile_valid", "tile_count", "tile_selected",
           "PauliDecompose", "PauliError", "load_library", "last_error", "ALGOS", "EXPORTS"]
