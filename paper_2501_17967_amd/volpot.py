"""Python binding of the C-ABI box code (libvolpot.so): argument marshalling only.

Every step of the volume potential runs in the HIP library; PyTorch supplies device memory
(``data_ptr()``) and the stream. There is no fallback: if the library is missing the import of
``lib()`` raises.

    plan = Plan(centres, levels)            # host arrays; validates the tree, uploads tables
    u = plan.apply(f)                       # f: cuda float64 (n_leaves, 16, 16) or (n, 256)
    fbar = plan.apply_adjoint(ubar)         # exact transpose
    u = volume_potential(f, plan)           # autograd: backward runs apply_adjoint
    lp = LayerPlan(centres, levels, nodes, weights, normals)   # glue layer potentials
    v = lp.apply(sigma, tau)                # S[sigma] - D[tau] at every leaf node
    pp = PointPlan(centres, levels, points) # u and grad u also at arbitrary points
    u, u_pts, grad = pp.apply_points(f)
    centres, levels = build_tree(f_of_points, eps, scale)   # adaptive quadtree on the GPU
    sp = StripPlan(gamma, gamma_t, q, n_r)  # strip solve (Sec. 4.3)
    v = sp.apply(f_at_sp_nodes)

Sign convention: u = int G f with G = -(1/2pi) log|x - y| (so -Lap u = f); the paper's v_bulk
(Sec. 4.2, eq. (vbulk)) is -u.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvolpot.so")

OK = 0
ERR_ARG, ERR_TREE, ERR_UNBALANCED, ERR_UNSUPPORTED, ERR_HIP, ERR_OOM, ERR_STATE = -1, -2, -3, -4, -5, -6, -7

EXPORTED = [
    "volpot_plan", "volpot_plan_forest", "volpot_apply", "volpot_apply_adjoint", "volpot_plan_info",
    "volpot_validate_tree", "volpot_nodes", "volpot_plan_destroy", "volpot_status_string",
    "volpot_set_timing", "volpot_stage_times", "volpot_plan_table", "volpot_near_relation",
    "volpot_plan_n_stages", "volpot_plan_stage", "volpot_autotune", "volpot_layer_plan", "volpot_layer_apply",
    "volpot_plan_points", "volpot_apply_points", "volpot_tree_create", "volpot_tree_pending", "volpot_tree_nodes",
    "volpot_tree_submit", "volpot_tree_leaves", "volpot_tree_destroy", "volpot_strip_plan", "volpot_strip_nodes",
    "volpot_strip_apply", "volpot_strip_destroy", "volpot_strip_apply_noalloc", "volpot_peak_mfma",
]

STAGE_KINDS = ["up", "down", "near", "loct", "adj_up", "adj_down", "adj_near", "adj_loct", "adj_sum", "nearc",
               "adj_nearc"]


class VolpotError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().volpot_status_string(code).decode() if _lib is not None else str(code)
        super().__init__("%s: %s (status %d)" % (what, msg, code))


class Options(ctypes.Structure):
    _fields_ = [("host_only", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("tile_leaf", ctypes.c_int32),
                ("tile_box", ctypes.c_int32), ("table_cache", ctypes.c_char_p), ("split_min", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("root_centre", ctypes.c_double * 2), ("root_halfwidth", ctypes.c_double),
                ("tile_leaf_exp", ctypes.c_int32), ("eps", ctypes.c_double), ("kchunk_leaf", ctypes.c_int32),
                ("dense_m2l", ctypes.c_int32), ("deterministic", ctypes.c_int32), ("dense_near", ctypes.c_int32)]


def _options(host_only=False, use_graph=False, tile_leaf=0, tile_box=0, table_cache=None, split_min=0, overlap=0,
             root_centre=(0.0, 0.0), root_halfwidth=0.0, tile_leaf_exp=0, eps=0.0, kchunk_leaf=0, dense_m2l=False,
             deterministic=False, dense_near=False):
    o = Options(int(host_only), int(use_graph), int(tile_leaf), int(tile_box),
                table_cache.encode() if table_cache else None, int(split_min), int(overlap))
    o.root_centre[0], o.root_centre[1] = float(root_centre[0]), float(root_centre[1])
    o.root_halfwidth = float(root_halfwidth)
    o.tile_leaf_exp = int(tile_leaf_exp)
    o.eps = float(eps)
    o.kchunk_leaf = int(kchunk_leaf)
    o.dense_m2l = int(bool(dense_m2l))
    o.deterministic = int(bool(deterministic))
    o.dense_near = int(bool(dense_near))
    return o


class Info(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int64), ("n_boxes", ctypes.c_int64), ("n_trees", ctypes.c_int64),
                ("max_level", ctypes.c_int32), ("order", ctypes.c_int32), ("n_reals", ctypes.c_int32),
                ("n_stages", ctypes.c_int32), ("pairs_near", ctypes.c_int64), ("pairs_v", ctypes.c_int64),
                ("pairs_w", ctypes.c_int64), ("pairs_x", ctypes.c_int64), ("n_m2m", ctypes.c_int64),
                ("n_l2l", ctypes.c_int64), ("n_s2m", ctypes.c_int64), ("n_l2t", ctypes.c_int64),
                ("flops_total", ctypes.c_double), ("flops_adjoint", ctypes.c_double),
                ("flops_kind", ctypes.c_double * 11), ("launches_kind", ctypes.c_int64 * 11),
                ("bytes_min", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("flops_issued_kind", ctypes.c_double * 11), ("n_layer_nodes", ctypes.c_int64),
                ("n_source_leaves", ctypes.c_int64), ("n_active_boxes", ctypes.c_int64), ("pairs_p2p", ctypes.c_int64),
                ("pairs_p2l", ctypes.c_int64), ("n_points", ctypes.c_int64), ("pairs_points", ctypes.c_int64),
                ("pairs_lowrank", ctypes.c_int64)]


class StageInfo(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("kind", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("kchunk", ctypes.c_int32), ("helper", ctypes.c_int32),
                ("n_tiles", ctypes.c_int64), ("n_segments", ctypes.c_int64), ("n_blocks", ctypes.c_int64),
                ("n_split_tiles", ctypes.c_int64), ("flops", ctypes.c_double), ("flops_issued", ctypes.c_double),
                ("inner", ctypes.c_int32), ("factored", ctypes.c_int32), ("n_chunks", ctypes.c_int64)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


def lib():
    """Load libvolpot.so (raises if it has not been built).

    PyTorch is imported first: it ships its own libamdhip64 / libhsa-runtime64, and the library
    must bind to that same HIP runtime (same soname) so that torch's streams and device pointers
    are valid in our launches. Loading the library first would pull in a second runtime.
    """
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (binds the process to torch's HIP runtime, see above)

        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvolpot.so is not built; run `python -m paper_2501_17967_amd.build` "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.volpot_plan.argtypes = [_dp, _ip, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(Options), ctypes.POINTER(_vp)]
        L.volpot_plan_forest.argtypes = [ctypes.c_int32, _lp, _dp, _ip, ctypes.c_int32, ctypes.POINTER(Options),
                                         ctypes.POINTER(_vp)]
        L.volpot_apply.argtypes = [_vp, _vp, _vp, _vp]
        L.volpot_apply_adjoint.argtypes = [_vp, _vp, _vp, _vp]
        L.volpot_plan_info.argtypes = [_vp, ctypes.POINTER(Info)]
        L.volpot_validate_tree.argtypes = [_dp, _ip, ctypes.c_int64, ctypes.c_int32, _lp]
        L.volpot_nodes.argtypes = [ctypes.c_int32, _dp, _dp]
        L.volpot_plan_destroy.argtypes = [_vp]
        L.volpot_plan_destroy.restype = None
        L.volpot_status_string.argtypes = [ctypes.c_int]
        L.volpot_status_string.restype = ctypes.c_char_p
        L.volpot_set_timing.argtypes = [_vp, ctypes.c_int32]
        L.volpot_stage_times.argtypes = [_vp, _dp, _lp, ctypes.c_int32]
        L.volpot_plan_table.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _dp, ctypes.c_int64]
        L.volpot_near_relation.argtypes = [ctypes.c_int32, _dp, _dp, _dp]
        L.volpot_plan_n_stages.argtypes = [_vp, ctypes.c_int32, _ip]
        L.volpot_autotune.argtypes = [ctypes.c_int32, _lp, _dp, _ip, ctypes.c_int32, ctypes.POINTER(Options),
                                      ctypes.c_char_p, ctypes.POINTER(Options), _dp]
        L.volpot_plan_stage.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(StageInfo)]
        L.volpot_layer_plan.argtypes = [_dp, _ip, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _dp, _dp, _dp,
                                        ctypes.POINTER(Options), ctypes.POINTER(_vp)]
        L.volpot_layer_apply.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.volpot_plan_points.argtypes = [_dp, _ip, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _dp,
                                         ctypes.POINTER(Options), ctypes.POINTER(_vp)]
        L.volpot_apply_points.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.volpot_tree_create.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(_vp)]
        L.volpot_tree_pending.argtypes = [_vp, _lp]
        L.volpot_tree_nodes.argtypes = [_vp, _vp, _vp]
        L.volpot_tree_submit.argtypes = [_vp, _vp, _vp]
        L.volpot_tree_leaves.argtypes = [_vp, _lp, _dp, _ip]
        L.volpot_tree_destroy.argtypes = [_vp]
        L.volpot_tree_destroy.restype = None
        L.volpot_strip_plan.argtypes = [ctypes.c_int32, ctypes.c_int32, _dp, _dp, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(_vp)]
        L.volpot_strip_nodes.argtypes = [_vp, _dp]
        L.volpot_strip_apply.argtypes = [_vp, _vp, _vp, _vp]
        L.volpot_strip_apply_noalloc.argtypes = [_vp, _vp, _vp, _vp]
        L.volpot_strip_destroy.argtypes = [_vp]
        L.volpot_strip_destroy.restype = None
        L.volpot_peak_mfma.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, _vp]
        _lib = L
    return _lib


def peak_mfma(blocks, iters, out, stream=None):
    """Launch the matrix-core rate kernel (volpot_peak_mfma) on `stream` (default: torch's
    current stream): blocks x 4 waves x iters x 8 FP64 MFMA of 2,048 flops; `out` is a float64
    CUDA tensor of 256 * blocks values (each thread's accumulator sum). Returns the flop count."""
    if out.dtype.itemsize != 8 or out.numel() < 256 * blocks or not out.is_cuda:
        raise ValueError("out must be a float64 device tensor of 256 * blocks values")
    _check(lib().volpot_peak_mfma(int(blocks), int(iters), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
           "volpot_peak_mfma")
    return float(blocks) * 4 * iters * 8 * 2048


def _check(code, what):
    if code != OK:
        raise VolpotError(code, what)


def _host_tree(centres, levels):
    c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 2))
    l = np.ascontiguousarray(np.asarray(levels, dtype=np.int32).reshape(-1))
    if c.shape[0] != l.shape[0]:
        raise ValueError("centres and levels differ in length")
    return c, l


def autotune(centres, levels, p=16, *, tree_offsets=None, cache=None, eps=0.0, dense_m2l=False, dense_near=False):
    """Fastest launch shape for this tree or forest on the current device (volpot_autotune):
    returns ({"tile_leaf", "tile_box", "split_min", "overlap", "tile_leaf_exp", "kchunk_leaf"}, ms per
    forward + adjoint apply). The candidates are timed at the expansion order that the far-field
    tolerance ``eps`` selects (0: the default), with the M2L and near-field forms that ``dense_m2l``
    and ``dense_near`` select. The result is looked up in / appended to the text file ``cache``
    when given."""
    c, l = _host_tree(centres, levels)
    off = np.ascontiguousarray(np.asarray([0, c.shape[0]] if tree_offsets is None else tree_offsets, dtype=np.int64))
    best = Options()
    base = _options(eps=eps, dense_m2l=dense_m2l, dense_near=dense_near)
    ms = ctypes.c_double(0.0)
    _check(lib().volpot_autotune(off.size - 1, off.ctypes.data_as(_lp), c.ctypes.data_as(_dp), l.ctypes.data_as(_ip), p,
                                 ctypes.byref(base), cache.encode() if cache else None, ctypes.byref(best),
                                 ctypes.byref(ms)),
           "volpot_autotune")
    return ({"tile_leaf": best.tile_leaf, "tile_box": best.tile_box, "split_min": best.split_min,
             "overlap": best.overlap, "tile_leaf_exp": best.tile_leaf_exp, "kchunk_leaf": best.kchunk_leaf}, ms.value)


def build_tree(f, eps, scale, min_level=0, max_level=24, p=16, stream=None):
    """Adaptive quadtree of f (Sec. 4.2.1) with 2:1 balance, built with the library's GPU tail
    test (volpot_tree_*). f maps a CUDA float64 tensor of points (n, 2) to n values (a CUDA
    tensor). Returns (centres (n, 2), levels (n,)) as NumPy arrays, ready for Plan."""
    import torch

    L = lib()
    h = _vp()
    _check(L.volpot_tree_create(p, float(eps), float(scale), int(min_level), int(max_level), ctypes.byref(h)),
           "volpot_tree_create")
    try:
        sh = _stream_handle(stream)
        n = ctypes.c_int64(0)
        while True:
            _check(L.volpot_tree_pending(h, ctypes.byref(n)), "volpot_tree_pending")
            if n.value == 0:
                break
            nodes = torch.empty((n.value * 256, 2), dtype=torch.float64, device="cuda")
            _check(L.volpot_tree_nodes(h, ctypes.c_void_p(nodes.data_ptr()), sh), "volpot_tree_nodes")
            vals = f(nodes)
            if not (isinstance(vals, torch.Tensor) and vals.is_cuda and vals.numel() == nodes.shape[0]):
                raise ValueError("f must return one CUDA value per point")
            vals = vals.to(torch.float64).contiguous()
            _check(L.volpot_tree_submit(h, ctypes.c_void_p(vals.data_ptr()), sh), "volpot_tree_submit")
        _check(L.volpot_tree_leaves(h, ctypes.byref(n), None, None), "volpot_tree_leaves")
        c = np.zeros((n.value, 2))
        lv = np.zeros(n.value, dtype=np.int32)
        _check(L.volpot_tree_leaves(h, ctypes.byref(n), c.ctypes.data_as(_dp), lv.ctypes.data_as(_ip)), "volpot_tree_leaves")
        return c, lv
    finally:
        L.volpot_tree_destroy(h)


class StripPlan:
    """Strip solve of Sec. 4.3 (volpot_strip_*): gamma and gamma_t are (n_panel, n_gl, 2) Gauss-Legendre
    nodes of corresponding panels of the boundary and of the fictitious curve; q and n_r the
    Chebyshev resolution along and across the strip. ``nodes`` (n_panel, n_r, q, 2) are where f is
    sampled; apply(f) returns v at those nodes."""

    def __init__(self, gamma, gamma_t, q=16, n_r=16):
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
        gt = np.ascontiguousarray(np.asarray(gamma_t, dtype=np.float64))
        if g.ndim != 3 or g.shape[2] != 2 or g.shape != gt.shape:
            raise ValueError("gamma and gamma_t must both be (n_panel, n_gl, 2)")
        self.shape = (g.shape[0], int(n_r), int(q))
        h = _vp()
        _check(lib().volpot_strip_plan(g.shape[0], g.shape[1], g.ctypes.data_as(_dp), gt.ctypes.data_as(_dp), int(q),
                                       int(n_r), ctypes.byref(h)), "volpot_strip_plan")
        self._h = h
        self.nodes = np.zeros(self.shape + (2,))
        _check(lib().volpot_strip_nodes(h, self.nodes.ctypes.data_as(_dp)), "volpot_strip_nodes")

    def apply(self, f, out=None, stream=None, noalloc=False):
        """v at the nodes. noalloc=True calls volpot_strip_apply_noalloc (work vectors in the
        library's static per-device array; ``out`` must then be given, so nothing is allocated)."""
        import torch

        if not (isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float64 and f.numel() == np.prod(self.shape)):
            raise TypeError("expected a CUDA float64 tensor of %d node values" % int(np.prod(self.shape)))
        if noalloc and (out is None or not f.is_contiguous()):
            raise ValueError("noalloc needs a contiguous f and a given out")
        f = f.contiguous()
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=f.device)
        fn = lib().volpot_strip_apply_noalloc if noalloc else lib().volpot_strip_apply
        _check(fn(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
               "volpot_strip_apply_noalloc" if noalloc else "volpot_strip_apply")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().volpot_strip_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def validate_tree(centres, levels, p=16):
    """(status, first bad leaf or -1) from the library's host-side tree check."""
    c, l = _host_tree(centres, levels)
    bad = ctypes.c_int64(-1)
    rc = lib().volpot_validate_tree(c.ctypes.data_as(_dp), l.ctypes.data_as(_ip), c.shape[0], p, ctypes.byref(bad))
    return rc, int(bad.value)


def nodes(p=16):
    t = np.zeros(p)
    w = np.zeros(p)
    _check(lib().volpot_nodes(p, t.ctypes.data_as(_dp), w.ctypes.data_as(_dp)), "volpot_nodes")
    return t, w


def near_relation(r):
    dx, dy, rho = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().volpot_near_relation(r, ctypes.byref(dx), ctypes.byref(dy), ctypes.byref(rho)), "volpot_near_relation")
    return dx.value, dy.value, rho.value


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A plan for one tree or, with ``tree_offsets``, a forest of independent trees."""

    def __init__(self, centres, levels, p=16, *, tree_offsets=None, host_only=False, use_graph=False,
                 tile_leaf=0, tile_box=0, table_cache=None, split_min=0, overlap=0, root_centre=(0.0, 0.0),
                 root_halfwidth=0.0, tile_leaf_exp=0, eps=0.0, kchunk_leaf=0, dense_m2l=False, deterministic=False,
                 dense_near=False):
        c, l = _host_tree(centres, levels)
        self.n_leaves = c.shape[0]
        opt = _options(host_only, use_graph, tile_leaf, tile_box, table_cache, split_min, overlap, root_centre,
                       root_halfwidth, tile_leaf_exp, eps, kchunk_leaf, dense_m2l, deterministic, dense_near)
        h = _vp()
        L = lib()
        if tree_offsets is None:
            rc = L.volpot_plan(c.ctypes.data_as(_dp), l.ctypes.data_as(_ip), self.n_leaves, p, ctypes.byref(opt), ctypes.byref(h))
            self.n_trees = 1
        else:
            off = np.ascontiguousarray(np.asarray(tree_offsets, dtype=np.int64))
            rc = L.volpot_plan_forest(off.size - 1, off.ctypes.data_as(_lp), c.ctypes.data_as(_dp), l.ctypes.data_as(_ip), p,
                                      ctypes.byref(opt), ctypes.byref(h))
            self.n_trees = off.size - 1
        _check(rc, "volpot_plan")
        self._h = h
        self.host_only = host_only

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().volpot_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = Info()
        _check(lib().volpot_plan_info(self._h, ctypes.byref(inf)), "volpot_plan_info")
        out = {}
        for name, _ in Info._fields_:
            v = getattr(inf, name)
            out[name] = {k: v[i] for i, k in enumerate(STAGE_KINDS)} if name in ("flops_kind", "launches_kind", "flops_issued_kind") else v
        return out

    def stages(self, adjoint=False):
        """The launches of one apply, in order: a list of dicts (name, kind, rows, tile, ...)."""
        L = lib()
        n = ctypes.c_int32(0)
        _check(L.volpot_plan_n_stages(self._h, int(adjoint), ctypes.byref(n)), "volpot_plan_n_stages")
        out = []
        for i in range(n.value):
            si = StageInfo()
            _check(L.volpot_plan_stage(self._h, int(adjoint), i, ctypes.byref(si)), "volpot_plan_stage")
            d = {k: getattr(si, k) for k, _ in StageInfo._fields_}
            d["name"] = si.name.decode()
            d["kind"] = STAGE_KINDS[si.kind]
            out.append(d)
        return out

    def table(self, kind, index=0):
        ne = self.info()["n_reals"]
        shape = {0: (256, 256), 1: (ne, 256), 2: (256, ne), 3: (256, 64), 4: (64, 256)}[kind]
        out = np.zeros(shape)
        _check(lib().volpot_plan_table(self._h, kind, index, out.ctypes.data_as(_dp), out.size), "volpot_plan_table")
        return out

    def set_timing(self, enable, kinds=None):
        """Time every stage kind (enable True), none (False), or only the named ``kinds``."""
        v = int(bool(enable))
        if enable and kinds is not None:
            v = sum(1 << (8 + STAGE_KINDS.index(k)) for k in kinds)
        _check(lib().volpot_set_timing(self._h, v), "volpot_set_timing")

    def stage_times(self):
        """{kind: (ms summed, launches)} since the last call (synchronises the timing events)."""
        ms = np.zeros(len(STAGE_KINDS))
        n = np.zeros(len(STAGE_KINDS), dtype=np.int64)
        _check(lib().volpot_stage_times(self._h, ms.ctypes.data_as(_dp), n.ctypes.data_as(_lp), len(STAGE_KINDS)),
               "volpot_stage_times")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGE_KINDS)}

    # ------------------------------------------------------------------
    def _prep(self, x, out):
        import torch

        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
            raise TypeError("expected a CUDA float64 tensor")
        if x.numel() != self.n_leaves * 256:
            raise ValueError("expected %d leaves x 256 values" % self.n_leaves)
        x = x.contiguous()
        if x.data_ptr() % 16:
            x = x.clone()
        if out is None:
            out = torch.empty_like(x)
        elif not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == x.numel()):
            raise ValueError("bad output tensor")
        return x, out

    def apply(self, f, out=None, stream=None):
        """u = A f (asynchronous on ``stream``, default the current stream)."""
        f, out = self._prep(f, out)
        _check(lib().volpot_apply(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  _stream_handle(stream)), "volpot_apply")
        return out

    def apply_adjoint(self, ubar, out=None, stream=None):
        """fbar = A^T ubar."""
        ubar, out = self._prep(ubar, out)
        _check(lib().volpot_apply_adjoint(self._h, ctypes.c_void_p(ubar.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          _stream_handle(stream)), "volpot_apply_adjoint")
        return out


class PointPlan(Plan):
    """A volume plan for one tree that also evaluates u and grad u at fixed points (m, 2); all of
    Plan's calls work on it."""

    def __init__(self, centres, levels, points, p=16, *, host_only=False, use_graph=False, tile_leaf=0, tile_box=0,
                 table_cache=None, split_min=0, overlap=0, root_centre=(0.0, 0.0), root_halfwidth=0.0, tile_leaf_exp=0):
        c, l = _host_tree(centres, levels)
        x = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 2))
        self.n_leaves = c.shape[0]
        self.n_points = x.shape[0]
        self.n_trees = 1
        opt = _options(host_only, use_graph, tile_leaf, tile_box, table_cache, split_min, overlap, root_centre,
                       root_halfwidth, tile_leaf_exp)
        h = _vp()
        _check(lib().volpot_plan_points(c.ctypes.data_as(_dp), l.ctypes.data_as(_ip), self.n_leaves, p, self.n_points,
                                        x.ctypes.data_as(_dp), ctypes.byref(opt), ctypes.byref(h)), "volpot_plan_points")
        self._h = h
        self.host_only = host_only

    def apply_points(self, f, out=None, grad=True, stream=None):
        """(u at the leaf nodes, u at the points (m,), grad u at the points (m, 2) or None)."""
        import torch

        f, out = self._prep(f, out)
        up = torch.empty(self.n_points, dtype=torch.float64, device=f.device)
        gp = torch.empty((self.n_points, 2), dtype=torch.float64, device=f.device) if grad else None
        _check(lib().volpot_apply_points(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(up.data_ptr() if self.n_points else 0),
                                         ctypes.c_void_p(gp.data_ptr()) if gp is not None and self.n_points else None,
                                         _stream_handle(stream)), "volpot_apply_points")
        return out, up, gp


class LayerPlan(Plan):
    """Evaluation of the glue layer potentials V = S[sigma] - D[tau] (Sec. 4.4) at every leaf node
    of one tree; the curve is given by quadrature nodes (m, 2), weights (m,) and unit normals (m, 2).
    Inspection (info, stages, timing) as for Plan; apply / apply_adjoint do not apply."""

    def __init__(self, centres, levels, nodes, weights, normals, p=16, *, host_only=False, use_graph=False,
                 tile_box=0, table_cache=None, split_min=0, overlap=0, root_centre=(0.0, 0.0), root_halfwidth=0.0):
        c, l = _host_tree(centres, levels)
        y = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(-1, 2))
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        n = np.ascontiguousarray(np.asarray(normals, dtype=np.float64).reshape(-1, 2))
        if not (y.shape[0] == w.shape[0] == n.shape[0]):
            raise ValueError("nodes, weights and normals differ in length")
        self.n_leaves = c.shape[0]
        self.n_nodes = y.shape[0]
        self.n_trees = 1
        opt = _options(host_only, use_graph, 0, tile_box, table_cache, split_min, overlap, root_centre, root_halfwidth)
        h = _vp()
        _check(lib().volpot_layer_plan(c.ctypes.data_as(_dp), l.ctypes.data_as(_ip), self.n_leaves, p, self.n_nodes,
                                       y.ctypes.data_as(_dp), w.ctypes.data_as(_dp), n.ctypes.data_as(_dp),
                                       ctypes.byref(opt), ctypes.byref(h)), "volpot_layer_plan")
        self._h = h
        self.host_only = host_only

    def apply(self, sigma, tau, out=None, stream=None):
        """V at every leaf node, (n_leaves, 256) float64 (asynchronous on ``stream``)."""
        import torch

        dens = []
        for x in (sigma, tau):
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
                raise TypeError("expected CUDA float64 densities")
            if x.numel() != self.n_nodes:
                raise ValueError("expected %d node values" % self.n_nodes)
            dens.append(x.contiguous())
        if out is None:
            out = torch.empty((self.n_leaves, 256), dtype=torch.float64, device=dens[0].device)
        elif not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == self.n_leaves * 256):
            raise ValueError("bad output tensor")
        ptr = [ctypes.c_void_p(d.data_ptr() if d.numel() else 0) for d in dens]
        _check(lib().volpot_layer_apply(self._h, ptr[0], ptr[1], ctypes.c_void_p(out.data_ptr()),
                                        _stream_handle(stream)), "volpot_layer_apply")
        return out

    def apply_adjoint(self, *args, **kwargs):
        raise VolpotError(ERR_STATE, "volpot_apply_adjoint")


def _autograd_cls():
    import torch

    class VolPot(torch.autograd.Function):
        """u = A f with dJ/df = A^T dJ/du from the hand-written adjoint kernels."""

        @staticmethod
        def forward(ctx, f, plan):
            ctx.plan = plan
            return plan.apply(f).view_as(f)

        @staticmethod
        def backward(ctx, grad):
            return ctx.plan.apply_adjoint(grad.contiguous()).view_as(grad), None

    return VolPot


_VolPot = None


def volume_potential(f, plan):
    """Differentiable u = A f (torch.autograd.Function backed by volpot_apply / _adjoint)."""
    global _VolPot
    if _VolPot is None:
        _VolPot = _autograd_cls()
    return _VolPot.apply(f, plan)
