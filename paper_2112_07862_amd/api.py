"""Python binding of libmembed: torch tensors supply device memory and the
stream; every step of the computation runs in the HIP library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


class MembedError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        self.name = L.STATUS_NAMES.get(status, str(status))
        super().__init__(f"{what}: {self.name} ({L.load().me_status_string(status).decode()})")


def _check(st: int, what: str) -> int:
    if st < 0:
        raise MembedError(st, what)
    return st


def _stream_ptr(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


_PRECISION = {"fp64": L.ME_FP64, "mixed": L.ME_MIXED}
_PRECOND = {"none": L.ME_PRECOND_NONE, "jacobi": L.ME_PRECOND_JACOBI,
            "chebyshev": L.ME_PRECOND_CHEBYSHEV}


_CHEB_OP = {"laplacian": L.ME_CHEB_LAPLACIAN, "full": L.ME_CHEB_FULL}
_ADDRESSING = {"auto": L.ME_ADDR_AUTO, "global": L.ME_ADDR_GLOBAL}
_ITERATES = {"fp32": L.ME_ITER_FP32, "fp16": L.ME_ITER_FP16}
_LAUNCH = {"auto": L.ME_LAUNCH_AUTO, "stream": L.ME_LAUNCH_STREAM, "graph": L.ME_LAUNCH_GRAPH}
_PRODUCT = {"fp64": L.ME_PRODUCT_FP64, "fp32": L.ME_PRODUCT_FP32}


def make_opts(precision="fp64", precond="chebyshev", max_iter=None, eps_max_iter=None,
              eps_tol=None, check_every=None, seed=None, cheb_degree=None,
              cheb_op=None, addressing=None, cheb_iterates=None, launch=None,
              cholqr_passes=None, product=None) -> L.MeOpts:
    o = L.MeOpts()
    L.load().me_opts_default(ctypes.byref(o))
    o.precision = _PRECISION[precision]
    o.precond = _PRECOND[precond]
    if max_iter is not None:
        o.max_iter = int(max_iter)
    if eps_max_iter is not None:
        o.eps_max_iter = int(eps_max_iter)
    if eps_tol is not None:
        o.eps_tol = float(eps_tol)
    if check_every is not None:
        o.check_every = int(check_every)
    if seed is not None:
        o.seed = int(seed)
    if cheb_degree is not None:
        o.cheb_degree = int(cheb_degree)
    if cheb_op is not None:
        o.cheb_op = _CHEB_OP[cheb_op]
    if addressing is not None:
        o.addressing = _ADDRESSING[addressing]
    if cheb_iterates is not None:
        o.cheb_iterates = _ITERATES[cheb_iterates]
    if launch is not None:
        o.launch = _LAUNCH[launch]
    if cholqr_passes is not None:
        o.cholqr_passes = int(cholqr_passes)
    if product is not None:
        o.product = _PRODUCT[product]
    return o


@dataclass
class DeviceCSR:
    n: int
    rowptr: torch.Tensor  # int64 [n+1]
    col: torch.Tensor     # int32 [nnz]
    val: torch.Tensor     # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def as_struct(self) -> L.MeCsr:
        return L.MeCsr(self.n, self.nnz, self.rowptr.data_ptr(), self.col.data_ptr(),
                       self.val.data_ptr())


def to_device(csr, device="cuda") -> DeviceCSR:
    """Uploads a host CSR (anything with n, rowptr, col, val)."""
    if isinstance(csr, DeviceCSR):
        return csr
    rp = torch.as_tensor(np.ascontiguousarray(csr.rowptr, dtype=np.int64)).to(device)
    col = torch.as_tensor(np.ascontiguousarray(csr.col, dtype=np.int32)).to(device)
    val = torch.as_tensor(np.ascontiguousarray(csr.val, dtype=np.float64)).to(device)
    return DeviceCSR(int(csr.n), rp, col, val)


class GraphOps:
    """Device-resident operators of one graph (T, Q, eps, mu, b, packed A)."""

    def __init__(self, handle: ctypes.c_void_p, n: int, info: L.MeInfo, status: int, csr):
        self._h = handle
        self.n = n
        self.build_info = info.as_dict()
        self.status = status
        self._csr = csr  # keep the input alive for the handle's lifetime
        lib = L.load()
        nn, nt, eps, mu, c = c_int64_(), c_int64_(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(lib.me_graph_ops_query(self._h, ctypes.byref(nn), ctypes.byref(nt), ctypes.byref(eps),
                                      ctypes.byref(mu), ctypes.byref(c)), "query")
        self.nnz_t = nt.value
        self.eps = eps.value
        self.mu = mu.value
        self.two_hop_disconnected = bool(c.value)
        self.device_bytes = int(lib.me_graph_ops_bytes(self._h))

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("GraphOps already closed")
        return self._h

    def export(self, stream=None) -> dict:
        dev = self._csr.rowptr.device
        n, nt = self.n, self.nnz_t
        out = dict(
            t_rowptr=torch.empty(n + 1, dtype=torch.int64, device=dev),
            t_col=torch.empty(max(nt, 1), dtype=torch.int32, device=dev),
            t_count=torch.empty(n, dtype=torch.int32, device=dev),
            d=torch.empty(n, dtype=torch.float64, device=dev),
            qdiag=torch.empty(n, dtype=torch.float64, device=dev),
            r=torch.empty(n, dtype=torch.float64, device=dev),
            b=torch.empty(n, dtype=torch.float64, device=dev),
        )
        _check(L.load().me_graph_ops_export(
            self.handle, _ptr(out["t_rowptr"]), _ptr(out["t_col"]), _ptr(out["t_count"]),
            _ptr(out["d"]), _ptr(out["qdiag"]), _ptr(out["r"]), _ptr(out["b"]),
            _stream_ptr(stream)), "export")
        out["t_col"] = out["t_col"][:nt]
        return out

    def order(self, stream=None) -> torch.Tensor:
        """Node order of the solver: perm[i] = caller's node of solver row i."""
        perm = torch.empty(self.n, dtype=torch.int32, device=self._csr.rowptr.device)
        _check(L.load().me_graph_ops_order(self.handle, _ptr(perm), _stream_ptr(stream)), "order")
        return perm

    def apply(self, which: str, X: torch.Tensor, stream=None) -> torch.Tensor:
        """Y = A X, Q X or B X (FP64 difference form)."""
        code = {"A": 0, "Q": 1, "B": 2}[which]
        X = X.contiguous()
        if X.dim() == 1:
            X = X[:, None]
        Y = torch.empty_like(X)
        _check(L.load().me_apply(self.handle, code, X.shape[1], _ptr(X), _ptr(Y),
                                 _stream_ptr(stream)), "apply")
        return Y

    def close(self):
        if self._h is not None:
            L.load().me_graph_ops_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def c_int64_():
    return ctypes.c_int64()


def knn_graph(points: torch.Tensor, k: int, workspace: torch.Tensor | None = None,
              stream=None):
    """Symmetric Gaussian-weighted kNN graph of `points` (n x dim float64,
    on the device) built on the GPU.  Returns (DeviceCSR, sigma)."""
    x = points.to(dtype=torch.float64).contiguous()
    if x.dim() != 2:
        raise ValueError("points must be n x dim")
    n, dim = int(x.shape[0]), int(x.shape[1])
    lib = L.load()
    cap = max(2 * n * int(k), 1)
    rp = torch.empty(n + 1, dtype=torch.int64, device=x.device)
    col = torch.empty(cap, dtype=torch.int32, device=x.device)
    val = torch.empty(cap, dtype=torch.float64, device=x.device)
    nnz, sigma = ctypes.c_int64(), ctypes.c_double()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(lib.me_knn_graph(_ptr(x), n, dim, int(k), _ptr(workspace), nbytes, _ptr(rp), _ptr(col),
                            _ptr(val), ctypes.byref(nnz), ctypes.byref(sigma),
                            _stream_ptr(stream)), "knn_graph")
    m = int(nnz.value)
    return DeviceCSR(n, rp, col[:m].clone(), val[:m].clone()), float(sigma.value)


def _ws_args(workspace):
    return _ptr(workspace), (0 if workspace is None else workspace.numel() * workspace.element_size())


def kmeans(X: torch.Tensor, C: int, u, max_iter: int = 100,
           workspace: torch.Tensor | None = None, stream=None):
    """k-means of the rows of X (n x K float64, device) into C clusters from
    the uniforms u (C values in [0, 1), the k-means++ draws).  Returns
    (labels int32 [n], centres [C, K], iterations)."""
    X = X.to(dtype=torch.float64).contiguous()
    n, K = int(X.shape[0]), int(X.shape[1])
    uu = (ctypes.c_double * int(C))(*[float(v) for v in u])
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    cen = torch.empty((int(C), K), dtype=torch.float64, device=X.device)
    it = ctypes.c_int()
    wp, wb = _ws_args(workspace)
    _check(L.load().me_kmeans(_ptr(X), n, K, int(C), uu, int(max_iter), wp, wb, _ptr(labels),
                              _ptr(cen), ctypes.byref(it), _stream_ptr(stream)), "kmeans")
    return labels, cen, it.value


def gmm(X: torch.Tensor, C: int, labels0: torch.Tensor, max_iter: int = 100, tol: float = 1e-6,
        workspace: torch.Tensor | None = None, stream=None):
    """EM for a full-covariance Gaussian mixture from the partition labels0.
    Returns (labels, weights [C], means [C, K], covs [C, K, K], loglik,
    iterations)."""
    X = X.to(dtype=torch.float64).contiguous()
    n, K = int(X.shape[0]), int(X.shape[1])
    l0 = labels0.to(dtype=torch.int32).contiguous()
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    w = torch.empty(int(C), dtype=torch.float64, device=X.device)
    mu = torch.empty((int(C), K), dtype=torch.float64, device=X.device)
    cov = torch.empty((int(C), K, K), dtype=torch.float64, device=X.device)
    ll, it = ctypes.c_double(), ctypes.c_int()
    wp, wb = _ws_args(workspace)
    _check(L.load().me_gmm(_ptr(X), n, K, int(C), _ptr(l0), int(max_iter), float(tol), wp, wb,
                           _ptr(labels), _ptr(w), _ptr(mu), _ptr(cov), ctypes.byref(ll),
                           ctypes.byref(it), _stream_ptr(stream)), "gmm")
    return labels, w, mu, cov, ll.value, it.value


def cluster_scores(classes: torch.Tensor, clusters: torch.Tensor, n_classes: int,
                   n_clusters: int, workspace: torch.Tensor | None = None, stream=None) -> dict:
    """RI, Precision, Purity and NMI of a clustering against known classes."""
    a = classes.to(dtype=torch.int32).contiguous()
    b = clusters.to(dtype=torch.int32).contiguous()
    out = (ctypes.c_double * 4)()
    wp, wb = _ws_args(workspace)
    _check(L.load().me_cluster_scores(_ptr(a), _ptr(b), int(a.numel()), int(n_classes),
                                      int(n_clusters), wp, wb, out, _stream_ptr(stream)),
           "cluster_scores")
    return {"RI": out[0], "Precision": out[1], "Purity": out[2], "NMI": out[3]}


def cluster_workspace_bytes(n: int, K: int, C: int) -> int:
    return int(L.load().me_cluster_workspace_bytes(int(n), int(K), int(C)))


def betweenness(csr, workspace: torch.Tensor | None = None, stream=None):
    """Betweenness centrality of every node (eq. (3), hop-count shortest
    paths) and its variance.  Returns (C_B tensor [n] float64, VBC)."""
    d = to_device(csr)
    cb = torch.empty(d.n, dtype=torch.float64, device=d.rowptr.device)
    v = ctypes.c_double()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(L.load().me_betweenness(ctypes.byref(d.as_struct()), _ptr(workspace), nbytes, _ptr(cb),
                                   ctypes.byref(v), _stream_ptr(stream)), "betweenness")
    return cb, float(v.value)


def betweenness_workspace_bytes(n: int) -> int:
    return int(L.load().me_betweenness_workspace_bytes(int(n)))


def knn_workspace_bytes(n: int, dim: int, k: int) -> int:
    return int(L.load().me_knn_workspace_bytes(int(n), int(dim), int(k)))


def build_workspace_bytes(csr, stream=None, **opts) -> int:
    """Device bytes build_graph_ops needs when given a workspace (an upper
    bound: the two-hop pattern is sized by W's degrees)."""
    dcsr = to_device(csr)
    o = make_opts(**opts)
    b = ctypes.c_size_t()
    _check(L.load().me_build_workspace_bytes(ctypes.byref(dcsr.as_struct()), ctypes.byref(o),
                                             _stream_ptr(stream), ctypes.byref(b)),
           "build_workspace_bytes")
    return int(b.value)


def build_graph_ops(csr, stream=None, workspace: torch.Tensor | None = None, **opts) -> GraphOps:
    """Builds the operators of one graph.  With `workspace` (a uint8 device
    tensor of at least build_workspace_bytes) every device array of the
    handle lives in it and the library allocates nothing; the tensor must
    outlive the handle (the handle keeps a reference)."""
    dcsr = to_device(csr)
    o = make_opts(**opts)
    h = ctypes.c_void_p()
    info = L.MeInfo()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    st = L.load().me_build_graph_ops(ctypes.byref(dcsr.as_struct()), ctypes.byref(o),
                                     _ptr(workspace), nbytes, _stream_ptr(stream),
                                     ctypes.byref(h), ctypes.byref(info))
    _check(st, "build_graph_ops")
    ops = GraphOps(h, dcsr.n, info, st, dcsr)
    ops._workspace = workspace
    return ops


def embed(graph, K: int, tol: float = 1e-6, X0: torch.Tensor | None = None,
          workspace: torch.Tensor | None = None, stream=None, **opts):
    """First K generalized eigenpairs of (A, B).  `graph` is a GraphOps or a
    CSR (built and released inside).  Returns (X [n, K] float64 B-orthonormal,
    lambda [K] float64 ascending, info dict)."""
    own = not isinstance(graph, GraphOps)
    ops = build_graph_ops(graph, stream=stream, **opts) if own else graph
    try:
        lib = L.load()
        o = make_opts(**opts)
        dev = ops._csr.rowptr.device
        need = int(lib.me_embed_workspace_bytes(ops.handle, int(K), ctypes.byref(o)))
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        X = torch.empty((ops.n, int(K)), dtype=torch.float64, device=dev)
        lam = torch.empty(int(K), dtype=torch.float64, device=dev)
        if X0 is not None:
            X0 = X0.to(device=dev, dtype=torch.float64).contiguous()
            if X0.shape != (ops.n, int(K)):
                raise ValueError("X0 must be n x K")
        info = L.MeInfo()
        st = lib.me_embed(ops.handle, int(K), float(tol), ctypes.byref(o), _ptr(X0),
                          _ptr(workspace), workspace.numel(), _ptr(X), _ptr(lam),
                          ctypes.byref(info), _stream_ptr(stream))
        _check(st, "embed")
        d = info.as_dict()
        d["status_name"] = L.STATUS_NAMES.get(st, str(st))
        d["ms_build"] = ops.build_info.get("ms_build", 0.0) if own else 0.0
        d["eps"] = ops.eps
        d["mu"] = ops.mu
        d["eps_iterations"] = ops.build_info.get("eps_iterations", 0)
        return X, lam, d
    finally:
        if own:
            ops.close()


def embed_batch_workspace_bytes(graphs, Ks, stream=None, **opts) -> int:
    """Device bytes embed_batch needs when given a workspace (an upper bound)."""
    G = len(graphs)
    if isinstance(Ks, int):
        Ks = [Ks] * G
    dcsrs = [to_device(g) for g in graphs]
    o = make_opts(**opts)
    Ws = (L.MeCsr * max(G, 1))(*[d.as_struct() for d in dcsrs])
    Kc = (ctypes.c_int * max(G, 1))(*[int(k) for k in Ks])
    b = ctypes.c_size_t()
    _check(L.load().me_embed_batch_workspace_bytes(G, Ws, Kc, ctypes.byref(o),
                                                   _stream_ptr(stream), ctypes.byref(b)),
           "embed_batch_workspace_bytes")
    return int(b.value)


def embed_batch(graphs, Ks, tol: float = 1e-6, stream=None,
                workspace: torch.Tensor | None = None, **opts):
    """Embeds many graphs in one batched solve.  `graphs`: CSRs (host or
    DeviceCSR); `Ks`: one K per graph (or a single int).  With `workspace` (a
    uint8 device tensor of at least embed_batch_workspace_bytes) the library
    allocates no device memory.  Returns a list of (X, lambda, info) per
    graph; graphs that failed carry info["status"] < 0 and X, lambda None.
    Raises only if the call as a whole is invalid."""
    lib = L.load()
    G = len(graphs)
    if isinstance(Ks, int):
        Ks = [Ks] * G
    if len(Ks) != G:
        raise ValueError("one K per graph")
    dcsrs = [to_device(g) for g in graphs]
    o = make_opts(**opts)
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    Xs = [torch.empty((d.n, int(k)), dtype=torch.float64, device=d.rowptr.device)
          for d, k in zip(dcsrs, Ks)]
    lams = [torch.empty(max(int(k), 1), dtype=torch.float64, device=d.rowptr.device)
            for d, k in zip(dcsrs, Ks)]
    Ws = (L.MeCsr * max(G, 1))(*[d.as_struct() for d in dcsrs])
    Kc = (ctypes.c_int * max(G, 1))(*[int(k) for k in Ks])
    Xp = (ctypes.c_void_p * max(G, 1))(*[x.data_ptr() for x in Xs])
    Lp = (ctypes.c_void_p * max(G, 1))(*[l.data_ptr() for l in lams])
    infos = (L.MeInfo * max(G, 1))()
    st = lib.me_embed_batch(G, Ws, Kc, float(tol), ctypes.byref(o), _ptr(workspace), nbytes,
                            Xp, Lp, infos, _stream_ptr(stream))
    if st in (-1, -7) and all(infos[i].status == 0 for i in range(G)):
        _check(st, "embed_batch")
    out = []
    for i in range(G):
        d = infos[i].as_dict()
        d["status_name"] = L.STATUS_NAMES.get(d["status"], str(d["status"]))
        if d["status"] < 0:
            out.append((None, None, d))
        else:
            out.append((Xs[i], lams[i][:int(Ks[i])], d))
    return out


def server_request_bytes(csr, K: int, stream=None) -> int:
    """Device footprint a Server charges a request (its reservation in a
    caller region)."""
    d = to_device(csr)
    b = ctypes.c_size_t()
    _check(L.load().me_server_request_bytes(ctypes.byref(d.as_struct()), int(K),
                                            _stream_ptr(stream), ctypes.byref(b)),
           "server_request_bytes")
    return int(b.value)


class Server:
    """Continuous-batching request loop (me_server_*): submit graphs at any
    time, call step() to advance every admitted solve by one round (and admit,
    retire and backfill), poll() for finished requests."""

    def __init__(self, mem_budget: int = 0, max_active: int = 256, stream=None,
                 workspace: torch.Tensor | None = None, **opts):
        """With `workspace` (a uint8 device tensor) every request's device
        memory is carved from it (mem_budget = its size) and the server
        allocates none; requests wait until their footprint fits."""
        lib = L.load()
        so = L.MeServerOpts()
        lib.me_server_opts_default(ctypes.byref(so))
        so.mem_budget = int(mem_budget)
        so.max_active = int(max_active)
        so.opts = make_opts(**opts)
        if workspace is not None:
            so.workspace = workspace.data_ptr()
            so.mem_budget = workspace.numel() * workspace.element_size()
        self._workspace = workspace
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib.me_server_create(ctypes.byref(so), _stream_ptr(stream), ctypes.byref(h)),
               "server_create")
        self._h = h
        self._pending = {}  # ticket -> (csr, W struct, X, lam, K)

    def submit(self, csr, K: int, tol: float = 1e-6) -> int:
        d = to_device(csr)
        X = torch.empty((d.n, int(K)), dtype=torch.float64, device=d.rowptr.device)
        lam = torch.empty(int(K), dtype=torch.float64, device=d.rowptr.device)
        W = d.as_struct()
        t = ctypes.c_int64()
        _check(L.load().me_server_submit(self._h, ctypes.byref(W), int(K), float(tol), _ptr(X),
                                         _ptr(lam), ctypes.byref(t)), "server_submit")
        self._pending[t.value] = (d, W, X, lam)
        return t.value

    def step(self) -> int:
        n = ctypes.c_int()
        _check(L.load().me_server_step(self._h, ctypes.byref(n)), "server_step")
        return n.value

    def poll(self, max_items: int = 1024):
        """Finished requests: list of (ticket, X, lambda, info); X, lambda are
        None for a failed request (info["status"] < 0)."""
        t = (ctypes.c_int64 * max_items)()
        inf = (L.MeInfo * max_items)()
        c = ctypes.c_int()
        _check(L.load().me_server_poll(self._h, t, inf, max_items, ctypes.byref(c)), "server_poll")
        out = []
        for q in range(c.value):
            d = inf[q].as_dict()
            d["status_name"] = L.STATUS_NAMES.get(d["status"], str(d["status"]))
            _, _, X, lam = self._pending.pop(t[q])
            out.append((t[q], X if d["status"] >= 0 else None, lam if d["status"] >= 0 else None, d))
        return out

    def close(self):
        if self._h is not None:
            L.load().me_server_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kernel_timing(kind: int) -> None:
    """Start timing one kernel kind (0 off, 1 SpMM of A, 2 Rayleigh-Ritz Gram,
    3 block combine, 4 Chebyshev preconditioner step); clears the totals."""
    _check(L.load().me_kernel_timing(int(kind)), "kernel_timing")


def step_form(block_width: int, range_: int, rows: int) -> int:
    """Form the run-time tuner kept for a kind of one-graph preconditioner
    step (0 halo-staged, 1 gathering, -1 not timed yet); range_ 1 = one-hop
    entries (embedding solve), 2 = two-hop entries (eps solve)."""
    return int(L.load().me_step_form(int(block_width), int(range_), int(rows)))


def step_form_reset() -> None:
    """Forgets every choice of the run-time tuner."""
    L.load().me_step_form_reset()


def kernel_timing_read() -> dict:
    n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(L.load().me_kernel_timing_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)),
           "kernel_timing_read")
    return {"launches": n.value, "total_ms": ms.value, "bytes": b.value}
