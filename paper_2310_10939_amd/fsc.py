"""Thin Python binding of libfsc (include/fsc.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Tensors are torch device tensors on the current HIP device; work is
queued on torch's current stream.  The library must be built
(`python -m paper_2310_10939_amd.build`); importing this module without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfsc.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"libfsc.so is not built ({_LIB_PATH}); run python -m paper_2310_10939_amd.build")
_lib = ctypes.CDLL(_LIB_PATH)

F64, F32, BF16 = 0, 1, 2
_DTYPES = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
_TORCH = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
_NAMES = {"f64": F64, "f32": F32, "bf16": BF16}


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("val_dtype", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("vec_dtype", ctypes.c_int32), ("kmeans_iters", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("renorm", ctypes.c_int32),
                ("x0", ctypes.c_void_p), ("sqnorm_trace", ctypes.c_void_p),
                ("rayleigh_trace", ctypes.c_void_p), ("tile_nnz", ctypes.c_int32),
                ("no_graph", ctypes.c_int32), ("return_y", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_nnz", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("xcd_order", ctypes.c_int32), ("unroll", ctypes.c_int32), ("slab_kb", ctypes.c_int32),
                ("slab_mode", ctypes.c_int32)]


_vp, _i32, _i64, _u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
_lib.fsc_create.argtypes = [ctypes.c_int, ctypes.POINTER(_vp)]
_lib.fsc_destroy.argtypes = [_vp]
_lib.fsc_destroy.restype = None
_lib.fsc_embed.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _i32, _u64, ctypes.POINTER(Opts), _vp, _vp]
_lib.fsc_cluster.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _i32, _i32, _u64, ctypes.POINTER(Opts), _vp, _vp,
                             _vp, _vp]
_lib.fsc_kmeans.argtypes = [_vp, _vp, _i32, _i64, _i32, _i32, _i32, _u64, _vp, _vp, _vp, _vp]
_lib.fsc_cluster_batched.argtypes = [_vp, _i32, ctypes.POINTER(Csr), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(_i32), _u64, ctypes.POINTER(Opts), _vp, _vp, _vp]
_lib.fsc_autotune.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _i32, ctypes.POINTER(Tuning), _vp]
_f = ctypes.c_float
_lib.fsc_mlp_param_count.restype = ctypes.c_int
_lib.fsc_filter_stats.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _i32, _i32, _u64, ctypes.POINTER(Opts), _vp, _vp,
                                  _vp, _vp, _vp]
_lib.fsc_mlp_forward.argtypes = [_vp, _vp, _i32, _vp, _vp, _vp]
_lib.fsc_mlp_loss_grad.argtypes = [_vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.fsc_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, _f, _i32, _vp]
_lib.fsc_mlp_train.argtypes = [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32, _f, _i32, _vp, _vp]
_lib.fsc_filter_embed.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _u64, _vp, _vp, _vp]
_lib.fsc_cluster_filtered.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _i32, _u64, _vp, _vp, _i32,
                                      ctypes.POINTER(Opts), _vp, _vp, _vp, ctypes.POINTER(_i32), _vp]
_lib.fsc_ari.argtypes = [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp]
_lib.fsc_nmi.argtypes = [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp]
_lib.fsc_knn.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp]
_lib.fsc_cluster_eigs.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _i32, _i32, _i32, _u64, ctypes.POINTER(Opts), _vp, _vp,
                                  _vp, _vp]
_lib.fsc_knn_graph.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp]
_lib.fsc_cluster_noalloc.argtypes = _lib.fsc_cluster.argtypes
_lib.fsc_cluster_pmk.argtypes = [_vp, ctypes.POINTER(Csr), _i32, _i32, _u64, ctypes.POINTER(Opts), _vp, _vp, _vp, _vp]
_lib.fsc_tuning_set.argtypes = [_vp, ctypes.POINTER(Tuning)]
_lib.fsc_timing_enable.argtypes = [_vp, ctypes.c_int]
_lib.fsc_timing_read.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)]
_lib.fsc_last_error.restype = ctypes.c_char_p
_lib.fsc_version.restype = ctypes.c_int

EXPORTS = ("fsc_create", "fsc_destroy", "fsc_embed", "fsc_cluster", "fsc_kmeans", "fsc_ari", "fsc_nmi",
           "fsc_cluster_batched", "fsc_autotune", "fsc_mlp_param_count", "fsc_filter_stats",
           "fsc_mlp_forward", "fsc_mlp_loss_grad", "fsc_mlp_adam", "fsc_mlp_train", "fsc_filter_embed",
           "fsc_cluster_filtered", "fsc_cluster_noalloc", "fsc_cluster_pmk", "fsc_cluster_eigs", "fsc_knn", "fsc_knn_graph",
           "fsc_tuning_set", "fsc_timing_enable", "fsc_timing_read", "fsc_last_error", "fsc_version")


class FscError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfsc error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise FscError(rc, _lib.fsc_last_error().decode())


_ctx_lock = threading.Lock()
_contexts = {}


def context(device=None):
    """The per-(thread, device) library context."""
    dev = torch.cuda.current_device() if device is None else int(device)
    key = (threading.get_ident(), dev)
    with _ctx_lock:
        c = _contexts.get(key)
        if c is None:
            p = _vp()
            _check(_lib.fsc_create(dev, ctypes.byref(p)))
            c = _contexts[key] = p
    return c


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _csr(indptr, indices, data):
    assert indptr.is_cuda and indptr.dtype == torch.int64 and indptr.is_contiguous()
    assert indices.is_cuda and indices.dtype == torch.int32 and indices.is_contiguous()
    g = Csr()
    g.n = indptr.numel() - 1
    g.nnz = indices.numel()
    g.row_ptr = indptr.data_ptr()
    g.col_idx = indices.data_ptr() if indices.numel() else None
    if data is not None:
        assert data.is_cuda and data.is_contiguous() and data.numel() == indices.numel()
        g.val = data.data_ptr()
        g.val_dtype = _DTYPES[data.dtype]
    else:
        g.val = None
        g.val_dtype = 0
    return g


def _opts(vec_dtype="f32", kmeans_iters=0, validate=False, renorm=False, x0=None, sqnorm=None,
          rayleigh=None, tile_nnz=0):
    o = Opts()
    o.vec_dtype = _NAMES[vec_dtype] if isinstance(vec_dtype, str) else int(vec_dtype)
    o.kmeans_iters = int(kmeans_iters)
    o.validate = int(validate)   # False/True -> 0/1; 2 adds the symmetry check
    o.renorm = int(bool(renorm))
    o.x0 = x0.data_ptr() if x0 is not None else None
    o.sqnorm_trace = sqnorm.data_ptr() if sqnorm is not None else None
    o.rayleigh_trace = rayleigh.data_ptr() if rayleigh is not None else None
    o.tile_nnz = int(tile_nnz)
    return o


def embed(indptr, indices, data, l, t, seed, vec_dtype="f32", x0=None, traces=False, renorm=False,
          validate=False, tile_nnz=0, return_y=False):
    """D^{-1/2} Y for l Gaussian start vectors and t PowerMethod steps
    (return_y=True: Y itself).

    Returns the n x l embedding (dtype per vec_dtype) and, with traces=True,
    also the FP64 (t+1) x l squared norms and t x l Rayleigh quotients.
    validate: 0/False none, 1/True the cheap checks, 2 also symmetry."""
    n = indptr.numel() - 1
    dev = indptr.device
    vd = _NAMES[vec_dtype]
    out = torch.empty((n, l), dtype=_TORCH[vd], device=dev)
    if x0 is not None:
        assert x0.dtype == torch.float64 and x0.is_contiguous() and x0.shape == (n, l)
    sq = torch.empty((t + 1, l), dtype=torch.float64, device=dev) if traces else None
    ray = torch.empty((max(t, 0), l), dtype=torch.float64, device=dev) if traces else None
    g = _csr(indptr, indices, data)
    o = _opts(vec_dtype, 0, validate, renorm, x0, sq, ray if (ray is not None and t > 0) else None, tile_nnz)
    o.return_y = int(bool(return_y))
    _check(_lib.fsc_embed(context(dev.index), ctypes.byref(g), l, t, seed, ctypes.byref(o), _ptr(out), _stream()))
    return (out, sq, ray) if traces else out


def cluster(indptr, indices, data, k, l, t, seed, kmeans_iters=30, vec_dtype="f32", x0=None, return_embedding=False,
            return_centres=False, validate=False, renorm=False, traces=False, tile_nnz=0, out=None):
    """FastSpectralCluster: labels (int32 [n]) of the k-way partition."""
    return _cluster(_lib.fsc_cluster, indptr, indices, data, k, l, t, seed, kmeans_iters, vec_dtype, x0,
                    return_embedding, return_centres, validate, renorm, traces, tile_nnz, out)


def cluster_noalloc(indptr, indices, data, k, l, t, seed, kmeans_iters=30, vec_dtype="f32", x0=None,
                    return_embedding=False, return_centres=False, validate=False, renorm=False, traces=False,
                    tile_nnz=0, out=None):
    """cluster() through fsc_cluster_noalloc: the library allocates no device
    memory (its workspace is a fixed scratch array of NOALLOC_MAX_BYTES per
    GPU); the outputs are allocated here unless `out` is given."""
    return _cluster(_lib.fsc_cluster_noalloc, indptr, indices, data, k, l, t, seed, kmeans_iters, vec_dtype, x0,
                    return_embedding, return_centres, validate, renorm, traces, tile_nnz, out)


NOALLOC_MAX_BYTES = 64 << 20


def _cluster(fn, indptr, indices, data, k, l, t, seed, kmeans_iters, vec_dtype, x0, return_embedding,
             return_centres, validate, renorm, traces, tile_nnz, out):
    n = indptr.numel() - 1
    dev = indptr.device
    vd = _NAMES[vec_dtype]
    labels = out if out is not None else torch.empty(n, dtype=torch.int32, device=dev)
    emb = torch.empty((n, l), dtype=_TORCH[vd], device=dev) if return_embedding else None
    cen = torch.empty((k, l), dtype=torch.float32, device=dev) if return_centres else None
    sq = torch.empty((t + 1, l), dtype=torch.float64, device=dev) if traces else None
    ray = torch.empty((max(t, 1), l), dtype=torch.float64, device=dev) if traces else None
    g = _csr(indptr, indices, data)
    o = _opts(vec_dtype, kmeans_iters, validate, renorm, x0, sq, ray, tile_nnz)
    _check(fn(context(dev.index), ctypes.byref(g), k, l, t, seed, ctypes.byref(o), _ptr(labels), _ptr(emb), _ptr(cen),
              _stream()))
    res = [labels]
    if return_embedding:
        res.append(emb)
    if return_centres:
        res.append(cen)
    if traces:
        res += [sq, ray[:t]]
    return res[0] if len(res) == 1 else tuple(res)


def cluster_pmk(indptr, indices, data, k, t, seed, kmeans_iters=30, vec_dtype="f32", x0=None, validate=False):
    """PM with k orthogonal vectors (k <= 8): (labels int32 [n], embedding
    FP32 n x k, the last step's singular values FP64 [k])."""
    n = indptr.numel() - 1
    dev = indptr.device
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    emb = torch.empty((n, k), dtype=torch.float32, device=dev)
    sv = torch.empty(k, dtype=torch.float64, device=dev)
    g = _csr(indptr, indices, data)
    o = _opts(vec_dtype, kmeans_iters, validate, False, x0)
    _check(_lib.fsc_cluster_pmk(context(dev.index), ctypes.byref(g), k, t, seed, ctypes.byref(o), _ptr(labels),
                                _ptr(emb), _ptr(sv), _stream()))
    return labels, emb, sv


def cluster_eigs(indptr, indices, data, k, m, cycles, steps, seed, kmeans_iters=30, vec_dtype="f32"):
    """Eigenvector baseline (m <= 8 leading eigenvectors by orthogonal
    iteration, cycles * steps steps): (labels int32 [n], embedding FP32
    n x m, eigenvalue estimates FP64 [m])."""
    n = indptr.numel() - 1
    dev = indptr.device
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    emb = torch.empty((n, m), dtype=torch.float32, device=dev)
    gam = torch.empty(m, dtype=torch.float64, device=dev)
    g = _csr(indptr, indices, data)
    o = _opts(vec_dtype, kmeans_iters)
    _check(_lib.fsc_cluster_eigs(context(dev.index), ctypes.byref(g), k, m, cycles, steps, seed, ctypes.byref(o),
                                 _ptr(labels), _ptr(emb), _ptr(gam), _stream()))
    return labels, emb, gam


def cluster_batched(graphs, ks, ls, ts, seed, kmeans_iters=30, return_embedding=False, use_graph=True):
    """The batched form: graphs is a list of (indptr, indices, data-or-None)
    device tensors; graph g uses seed + g.  Returns the concatenated int32
    labels (and the concatenated FP32 embeddings) plus the per-graph offsets."""
    G = len(graphs)
    dev = graphs[0][0].device
    arr = (Csr * G)()
    ns = []
    for g, (ip, ix, d) in enumerate(graphs):
        arr[g] = _csr(ip, ix, d)
        ns.append(ip.numel() - 1)
    off = [0]
    eoff = [0]
    for g in range(G):
        off.append(off[-1] + ns[g])
        eoff.append(eoff[-1] + ns[g] * int(ls[g]))
    labels = torch.empty(off[-1], dtype=torch.int32, device=dev)
    emb = torch.empty(eoff[-1], dtype=torch.float32, device=dev) if return_embedding else None
    K = (_i32 * G)(*[int(x) for x in ks])
    L = (_i32 * G)(*[int(x) for x in ls])
    T = (_i32 * G)(*[int(x) for x in ts])
    o = _opts("f32", kmeans_iters)
    o.no_graph = 0 if use_graph else 1
    _check(_lib.fsc_cluster_batched(context(dev.index), G, arr, K, L, T, seed, ctypes.byref(o), _ptr(labels),
                                    _ptr(emb), _stream()))
    return (labels, emb, off, eoff) if return_embedding else (labels, off)


def autotune(indptr, indices, data, l, steps=5):
    """Times the candidate launch shapes of the sparse product on this graph,
    keeps the fastest as the context default (and for the graph's degree
    class in the batched form) and returns it."""
    g = _csr(indptr, indices, data)
    t = Tuning()
    _check(_lib.fsc_autotune(context(indptr.device.index), ctypes.byref(g), l, steps, ctypes.byref(t), _stream()))
    return {"tile_nnz": t.tile_nnz, "blocks_per_cu": t.blocks_per_cu, "xcd_order": t.xcd_order, "unroll": t.unroll,
            "slab_kb": t.slab_kb, "slab_mode": t.slab_mode}


# ---------------------------------------------------------------------------
# The learned polynomial-filter form
# ---------------------------------------------------------------------------
def mlp_param_count():
    return _lib.fsc_mlp_param_count()


def filter_stats(indptr, indices, data, k, l, t, seed, kmeans_iters=30):
    """Training statistics of one graph: (features float32[9], within
    float64[9,9], total float64[9,9], labels int32[n]) device tensors; the
    labels are the plain method's."""
    dev = indptr.device
    n = indptr.numel() - 1
    feat = torch.empty(9, dtype=torch.float32, device=dev)
    W = torch.empty((9, 9), dtype=torch.float64, device=dev)
    T = torch.empty((9, 9), dtype=torch.float64, device=dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    g = _csr(indptr, indices, data)
    o = _opts(kmeans_iters=kmeans_iters)
    _check(_lib.fsc_filter_stats(context(dev.index), ctypes.byref(g), k, l, t, seed, ctypes.byref(o), _ptr(feat),
                                 _ptr(W), _ptr(T), _ptr(labels), _stream()))
    return feat, W, T, labels


def mlp_forward(params, feats):
    feats = feats.contiguous()
    out = torch.empty((feats.shape[0], 8), dtype=torch.float32, device=feats.device)
    _check(_lib.fsc_mlp_forward(context(feats.device.index), _ptr(params), feats.shape[0], _ptr(feats), _ptr(out),
                                _stream()))
    return out


def mlp_loss_grad(params, feats, W, T):
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float64, device=params.device)
    _check(_lib.fsc_mlp_loss_grad(context(params.device.index), _ptr(params), feats.shape[0], _ptr(feats), _ptr(W),
                                  _ptr(T), _ptr(grad), _ptr(loss), _stream()))
    return loss, grad


def mlp_adam(params, m, v, grad, lr, step):
    _check(_lib.fsc_mlp_adam(context(params.device.index), _ptr(params), _ptr(m), _ptr(v), _ptr(grad), lr, step,
                             _stream()))


def mlp_train(params, m, v, feats, W, T, steps, lr, first_step=1):
    """`steps` full-batch Adam steps on the device; returns the loss trace."""
    trace = torch.empty(steps, dtype=torch.float64, device=params.device)
    _check(_lib.fsc_mlp_train(context(params.device.index), _ptr(params), _ptr(m), _ptr(v), feats.shape[0],
                              _ptr(feats), _ptr(W), _ptr(T), steps, lr, first_step, _ptr(trace), _stream()))
    return trace


def filter_embed(indptr, indices, data, l, seed, coeffs):
    """D^{-1/2} p(M) X0 with coefficients c_1..c_8 (float32[8] device)."""
    n = indptr.numel() - 1
    out = torch.empty((n, l), dtype=torch.float32, device=indptr.device)
    g = _csr(indptr, indices, data)
    _check(_lib.fsc_filter_embed(context(indptr.device.index), ctypes.byref(g), l, seed, _ptr(coeffs), _ptr(out),
                                 _stream()))
    return out


def cluster_filtered(indptr, indices, data, k, l, seed, params=None, coeffs=None, fallback_t=0, kmeans_iters=30,
                     diagnostics=False):
    """The learned form: returns (labels, coefficients used, used_fallback)
    and, with diagnostics=True, the device double[4] (rho_f, rho_8,
    normalised k-means cost, flag)."""
    n = indptr.numel() - 1
    dev = indptr.device
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    cout = torch.empty(8, dtype=torch.float32, device=dev)
    diag = torch.empty(4, dtype=torch.float64, device=dev)
    used = _i32(0)
    g = _csr(indptr, indices, data)
    o = _opts("f32", kmeans_iters)
    _check(_lib.fsc_cluster_filtered(context(dev.index), ctypes.byref(g), k, l, seed, _ptr(params), _ptr(coeffs),
                                     fallback_t, ctypes.byref(o), _ptr(labels), _ptr(cout), _ptr(diag),
                                     ctypes.byref(used), _stream()))
    if diagnostics:
        return labels, cout, bool(used.value), diag
    return labels, cout, bool(used.value)


def knn(X, k):
    """Exact k nearest neighbours (k <= 16) of the rows of a contiguous FP32
    device matrix: (indices int32 [n, k], squared distances FP32 [n, k])."""
    assert X.dtype == torch.float32 and X.is_contiguous() and X.dim() == 2
    n, dim = X.shape
    nbr = torch.empty((n, k), dtype=torch.int32, device=X.device)
    dist = torch.empty((n, k), dtype=torch.float32, device=X.device)
    _check(_lib.fsc_knn(context(X.device.index), _ptr(X), n, dim, k, _ptr(nbr), _ptr(dist), _stream()))
    return nbr, dist


def knn_graph(X, k):
    """The symmetrised kNN graph of the rows of a contiguous FP32 device
    matrix: device (indptr int64 [n+1], indices int32, weights FP32), trimmed
    to the stored entries."""
    assert X.dtype == torch.float32 and X.is_contiguous() and X.dim() == 2
    n, dim = X.shape
    indptr = torch.empty(n + 1, dtype=torch.int64, device=X.device)
    indices = torch.empty(2 * n * k, dtype=torch.int32, device=X.device)
    weights = torch.empty(2 * n * k, dtype=torch.float32, device=X.device)
    _check(_lib.fsc_knn_graph(context(X.device.index), _ptr(X), n, dim, k, _ptr(indptr), _ptr(indices),
                              _ptr(weights), _stream()))
    nnz = int(indptr[-1])
    return indptr, indices[:nnz], weights[:nnz]


def kmeans(points, k, iters, seed, eligible=None):
    """k-means++ then `iters` Lloyd steps on the rows of `points` (n x l,
    float32/float64).  Returns (labels int32 [n], centres float32 [k, l])."""
    assert points.is_cuda and points.dim() == 2 and points.is_contiguous()
    n, l = points.shape
    labels = torch.empty(n, dtype=torch.int32, device=points.device)
    cen = torch.empty((k, l), dtype=torch.float32, device=points.device)
    if eligible is not None:
        assert eligible.dtype == torch.uint8 and eligible.is_contiguous() and eligible.numel() == n
    _check(_lib.fsc_kmeans(context(points.device.index), _ptr(points), _DTYPES[points.dtype], n, l, k, iters, seed,
                           _ptr(eligible), _ptr(labels), _ptr(cen), _stream()))
    return labels, cen


def ari(a, b, ka, kb):
    """Adjusted Rand index of two int32 device labelings (an FP64 0-d tensor)."""
    out = torch.empty((), dtype=torch.float64, device=a.device)
    _check(_lib.fsc_ari(context(a.device.index), _ptr(a), _ptr(b), a.numel(), ka, kb, _ptr(out), _stream()))
    return out


def nmi(a, b, ka, kb):
    """Normalised mutual information (arithmetic-mean normalisation) of two
    int32 device labelings (an FP64 0-d tensor)."""
    out = torch.empty((), dtype=torch.float64, device=a.device)
    _check(_lib.fsc_nmi(context(a.device.index), _ptr(a), _ptr(b), a.numel(), ka, kb, _ptr(out), _stream()))
    return out


def tuning(tile_nnz=0, blocks_per_cu=0, xcd_order=0, unroll=0, slab_kb=0, slab_mode=0, device=None):
    """Sets the sparse-product launch shape (0 keeps a field; slab_kb < 0
    turns the column-slab form off; slab_mode 1 phases, 2 per-XCD, 4 waves,
    3 automatic) and returns the current one as a dict (xcd_order: 1 contiguous
    per XCD, 2 round robin)."""
    t = Tuning(tile_nnz, blocks_per_cu, xcd_order, unroll, slab_kb, slab_mode)
    _check(_lib.fsc_tuning_set(context(device), ctypes.byref(t)))
    return {"tile_nnz": t.tile_nnz, "blocks_per_cu": t.blocks_per_cu, "xcd_order": t.xcd_order,
            "unroll": t.unroll, "slab_kb": t.slab_kb, "slab_mode": t.slab_mode}


def timing_enable(on=True, device=None):
    """Brackets every sparse-product launch with HIP events (see fsc.h)."""
    _check(_lib.fsc_timing_enable(context(device), int(bool(on))))


def timing_read(device=None):
    """(launches, total_ms) of the sparse-product launches timed so far."""
    n = _i64()
    ms = ctypes.c_double()
    _check(_lib.fsc_timing_read(context(device), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def version():
    v = _lib.fsc_version()
    return (v >> 16, v & 0xFFFF)
