"""ctypes binding of libqsd (include/qsd.h).  Argument marshalling only: every step of a
transposition runs in the library's HIP kernels.  PyTorch supplies device memory and
streams.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsd.so")
MODEL_PATH = os.path.join(HERE, "selector", "selector_model.bin")  # the trained schedule selector

QSD_OK = 0
STATUS = {0: "ok", 1: "null", 2: "bad order", 3: "bad extent", 4: "too large", 5: "unsorted",
          6: "coordinate range", 7: "workspace", 8: "unsupported", 9: "hip", 10: "device"}
QSD_I32, QSD_I64 = 0, 1
QSD_F32, QSD_F64 = 0, 1
SCHED = {"auto": 0, "minimal": 1, "top2": 2, "lsd": 3}
QSD_SCHED_TOPK = 16  # + K: Top-K-sadilla with that K


def sched_code(sched):
    """Schedule code from a name ("minimal", "top2", "lsd", "auto", "topk<K>") or an int."""
    if not isinstance(sched, str):
        return int(sched)
    if sched.startswith("topk"):
        return QSD_SCHED_TOPK + int(sched[4:])
    return SCHED[sched]
QSD_VALIDATE = 1
QSD_KEEP_BUCKETS = 2
QSD_ERR_WORKSPACE = 7
QSD_NOALLOC_MAX_WORKSPACE = 64 << 20  # as declared in qsd.h
MAX_ORDER = 8


class QsdError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: qsd status {code} ({STATUS.get(code, '?')})")


class qsd_desc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("extents", ctypes.POINTER(ctypes.c_int64)), ("crd_type", ctypes.c_int),
                ("val_type", ctypes.c_int), ("in_order", ctypes.POINTER(ctypes.c_int32)),
                ("out_order", ctypes.POINTER(ctypes.c_int32)), ("flags", ctypes.c_uint32)]


class qsd_batch_io(ctypes.Structure):
    _fields_ = [("in_crd", ctypes.c_void_p * 8), ("in_val", ctypes.c_void_p),
                ("out_crd", ctypes.c_void_p * 8), ("out_val", ctypes.c_void_p)]


class qsd_tuning(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int32), ("radix_bits", ctypes.c_int32), ("small_cap", ctypes.c_int32)]


class qsd_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None
_VP = ctypes.c_void_p


def load():
    """Load libqsd.so (raises when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    lib.qsd_plan.argtypes = [ctypes.POINTER(qsd_desc), ctypes.c_int, ctypes.POINTER(_VP)]
    lib.qsd_plan_destroy.argtypes = [_VP]
    lib.qsd_plan_destroy.restype = None
    lib.qsd_plan_workspace.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_plan_describe.argtypes = [_VP, ctypes.c_char_p, ctypes.c_size_t]
    lib.qsd_transpose.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(_VP), _VP, ctypes.POINTER(_VP), _VP,
                                  _VP, ctypes.c_size_t, _VP]
    lib.qsd_transpose_noalloc.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(_VP), _VP, ctypes.POINTER(_VP), _VP,
                                          _VP]
    lib.qsd_csf_transpose_workspace.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_csf_transpose.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP,
                                      ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP, _VP, _VP, ctypes.c_size_t, _VP]
    lib.qsd_csf_workspace.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_pack_csf.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                 ctypes.POINTER(_VP), _VP, _VP, ctypes.c_size_t, _VP]
    lib.qsd_device_status.argtypes = [_VP, _VP, ctypes.POINTER(ctypes.c_uint32)]
    lib.qsd_profile_start.argtypes = []
    lib.qsd_profile_stop.argtypes = [ctypes.POINTER(qsd_kernel_stat), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]
    lib.qsd_status_str.argtypes = [ctypes.c_int]
    lib.qsd_status_str.restype = ctypes.c_char_p
    lib.qsd_batch_plan.argtypes = [ctypes.POINTER(qsd_desc), ctypes.c_int32, ctypes.POINTER(_VP)]
    lib.qsd_batch_destroy.argtypes = [_VP]
    lib.qsd_batch_destroy.restype = None
    lib.qsd_batch_set_tuning.argtypes = [_VP, ctypes.POINTER(qsd_tuning)]
    lib.qsd_batch_get_tuning.argtypes = [_VP, ctypes.POINTER(qsd_tuning)]
    lib.qsd_batch_workspace.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_batch_workspace_max.argtypes = [_VP, ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_batch_bind.argtypes = [_VP, ctypes.POINTER(qsd_batch_io), _VP, ctypes.c_size_t, _VP]
    lib.qsd_batch_transpose.argtypes = [_VP, _VP, ctypes.c_size_t, _VP]
    lib.qsd_batch_tune.argtypes = [_VP, ctypes.POINTER(qsd_batch_io), _VP, ctypes.c_size_t, _VP, ctypes.c_int32,
                                   ctypes.POINTER(qsd_tuning), ctypes.POINTER(ctypes.c_float)]
    lib.qsd_batch_tune_key.argtypes = [_VP, ctypes.c_char_p, ctypes.c_size_t]
    lib.qsd_batch_tune_cached.argtypes = [_VP, ctypes.POINTER(qsd_batch_io), _VP, ctypes.c_size_t, _VP, ctypes.c_int32,
                                          ctypes.c_char_p, ctypes.POINTER(qsd_tuning), ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.qsd_batch_graph.argtypes = [_VP, _VP, ctypes.c_size_t, ctypes.POINTER(_VP)]
    lib.qsd_graph_launch.argtypes = [_VP, _VP]
    lib.qsd_graph_destroy.argtypes = [_VP]
    lib.qsd_graph_destroy.restype = None
    F = ctypes.POINTER(ctypes.c_float)
    U32 = ctypes.POINTER(ctypes.c_uint32)
    lib.qsd_select_workspace.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_feature_counts.argtypes = [ctypes.POINTER(qsd_desc), ctypes.POINTER(_VP), _VP, ctypes.c_size_t, _VP,
                                       U32, U32, U32]
    lib.qsd_features.argtypes = [ctypes.POINTER(qsd_desc), ctypes.POINTER(_VP), _VP, ctypes.c_size_t, _VP, F]
    lib.qsd_mlp_init.argtypes = [ctypes.c_uint64, F]
    lib.qsd_mlp_forward.argtypes = [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP]
    lib.qsd_mlp_backward_workspace.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_mlp_backward.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t,
                                     _VP]
    lib.qsd_mlp_adam.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, _VP]
    lib.qsd_mlp_train_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    lib.qsd_mlp_train.argtypes = [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                  ctypes.c_uint64, _VP, ctypes.c_size_t, _VP, F]
    lib.qsd_model_create.argtypes = [F, ctypes.c_float, ctypes.c_int64, ctypes.POINTER(_VP)]
    lib.qsd_model_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(_VP)]
    lib.qsd_model_destroy.argtypes = [_VP]
    lib.qsd_model_destroy.restype = None
    lib.qsd_select.argtypes = [_VP, ctypes.POINTER(qsd_desc), ctypes.POINTER(_VP), _VP, ctypes.c_size_t, _VP,
                               ctypes.POINTER(ctypes.c_int32), F]
    lib.qsd_plan_auto.argtypes = [_VP, ctypes.POINTER(qsd_desc), ctypes.POINTER(_VP), _VP, ctypes.c_size_t, _VP,
                                  ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int32)]
    lib.qsd_candidate.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint32)]
    I32 = ctypes.POINTER(ctypes.c_int32)
    lib.qsd_candidate_terms.argtypes = [ctypes.POINTER(qsd_desc), I32, I32, I32]
    for name in ("qsd_select_workspace", "qsd_feature_counts", "qsd_features", "qsd_mlp_init", "qsd_mlp_forward",
                 "qsd_mlp_backward_workspace", "qsd_mlp_backward", "qsd_mlp_adam", "qsd_mlp_train_workspace",
                 "qsd_mlp_train", "qsd_model_create", "qsd_model_load", "qsd_select", "qsd_plan_auto",
                 "qsd_candidate", "qsd_candidate_terms"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("qsd_plan", "qsd_plan_workspace", "qsd_plan_describe", "qsd_transpose", "qsd_transpose_noalloc",
                 "qsd_csf_workspace", "qsd_pack_csf", "qsd_device_status", "qsd_profile_start",
                 "qsd_csf_transpose_workspace", "qsd_csf_transpose",
                 "qsd_profile_stop", "qsd_batch_plan", "qsd_batch_set_tuning", "qsd_batch_get_tuning",
                 "qsd_batch_workspace", "qsd_batch_workspace_max", "qsd_batch_bind", "qsd_batch_transpose",
                 "qsd_batch_tune", "qsd_batch_tune_key", "qsd_batch_tune_cached", "qsd_batch_graph",
                 "qsd_graph_launch"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code, where):
    if code != QSD_OK:
        raise QsdError(code, where)


def _ptrs(seq):
    arr = (_VP * MAX_ORDER)()
    for i, p in enumerate(seq):
        arr[i] = p
    return arr


# ---------------------------------------------------------------- raw C-ABI mirrors

def qsd_plan(order, nnz, extents, crd_type, val_type, in_order, out_order, sched="minimal", flags=0):
    """Returns an opaque plan handle (int)."""
    lib = load()
    d, _keep = _desc(order, nnz, extents, crd_type, val_type, in_order, out_order, flags)
    h = _VP()
    _check(lib.qsd_plan(ctypes.byref(d), sched_code(sched),
                        ctypes.byref(h)), "qsd_plan")
    return h.value


def _desc(order, nnz, extents, crd_type, val_type, in_order, out_order, flags=0):
    r = int(order)
    ext = (ctypes.c_int64 * max(r, 1))(*[int(x) for x in extents])
    ino = (ctypes.c_int32 * max(r, 1))(*[int(x) for x in in_order])
    outo = (ctypes.c_int32 * max(r, 1))(*[int(x) for x in out_order])
    return qsd_desc(r, int(nnz), ext, int(crd_type), int(val_type), ino, outo, int(flags)), (ext, ino, outo)


def qsd_plan_destroy(plan):
    load().qsd_plan_destroy(plan)


def qsd_plan_workspace(plan):
    n = ctypes.c_size_t()
    _check(load().qsd_plan_workspace(plan, ctypes.byref(n)), "qsd_plan_workspace")
    return n.value


def qsd_plan_describe(plan):
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().qsd_plan_describe(plan, buf, len(buf)), "qsd_plan_describe")
    return buf.value.decode()


def qsd_transpose(plan, nnz, in_crd, in_val, out_crd, out_val, ws, ws_bytes, stream):
    """in_crd/out_crd: sequences of device pointers (ints); others device pointers/ints."""
    _check(load().qsd_transpose(plan, int(nnz), _ptrs(in_crd), in_val, _ptrs(out_crd), out_val,
                                ws, int(ws_bytes), stream), "qsd_transpose")


def qsd_transpose_noalloc(plan, nnz, in_crd, in_val, out_crd, out_val, stream):
    """qsd_transpose on the library's fixed per-GPU workspace (no allocation)."""
    _check(load().qsd_transpose_noalloc(plan, int(nnz), _ptrs(in_crd), in_val, _ptrs(out_crd), out_val, stream),
           "qsd_transpose_noalloc")


def qsd_csf_workspace(plan):
    n = ctypes.c_size_t()
    _check(load().qsd_csf_workspace(plan, ctypes.byref(n)), "qsd_csf_workspace")
    return n.value


def qsd_pack_csf(plan, nnz, sorted_crd, pos, crd, fiber_counts, ws, ws_bytes, stream):
    _check(load().qsd_pack_csf(plan, int(nnz), _ptrs(sorted_crd), _ptrs(pos), _ptrs(crd), fiber_counts,
                               ws, int(ws_bytes), stream), "qsd_pack_csf")


def qsd_csf_transpose_workspace(plan):
    n = ctypes.c_size_t()
    _check(load().qsd_csf_transpose_workspace(plan, ctypes.byref(n)), "qsd_csf_transpose_workspace")
    return n.value


def qsd_csf_transpose(plan, nnz, in_pos, in_crd, in_val, out_pos, out_crd, out_val, fiber_counts, ws, ws_bytes,
                      stream):
    _check(load().qsd_csf_transpose(plan, int(nnz), _ptrs(in_pos), _ptrs(in_crd), in_val, _ptrs(out_pos),
                                    _ptrs(out_crd), out_val, fiber_counts, ws, int(ws_bytes), stream),
           "qsd_csf_transpose")


def qsd_device_status(ws, stream):
    code = ctypes.c_uint32()
    _check(load().qsd_device_status(ws, stream, ctypes.byref(code)), "qsd_device_status")
    return code.value


def qsd_profile_start():
    _check(load().qsd_profile_start(), "qsd_profile_start")


def qsd_profile_stop():
    """{kind: (launches, total_ms, algorithmic_bytes)} of the launches since qsd_profile_start."""
    out = (qsd_kernel_stat * 32)()
    n = ctypes.c_int32()
    _check(load().qsd_profile_stop(out, 32, ctypes.byref(n)), "qsd_profile_stop")
    return {out[i].name.decode(): (out[i].launches, out[i].total_ms, out[i].bytes) for i in range(n.value)}


def qsd_batch_plan(tensors):
    """tensors: sequence of (order, nnz, extents, crd_type, val_type, in_order, out_order).
    Returns an opaque batch handle (int)."""
    keep = []
    arr = (qsd_desc * max(len(tensors), 1))()
    for i, t in enumerate(tensors):
        d, k = _desc(*t)
        arr[i] = d
        keep.append(k)
    h = _VP()
    _check(load().qsd_batch_plan(arr, len(tensors), ctypes.byref(h)), "qsd_batch_plan")
    return h.value


def qsd_batch_destroy(batch):
    load().qsd_batch_destroy(batch)


def qsd_batch_set_tuning(batch, items, radix_bits, small_cap):
    t = qsd_tuning(int(items), int(radix_bits), int(small_cap))
    _check(load().qsd_batch_set_tuning(batch, ctypes.byref(t)), "qsd_batch_set_tuning")


def qsd_batch_get_tuning(batch):
    t = qsd_tuning()
    _check(load().qsd_batch_get_tuning(batch, ctypes.byref(t)), "qsd_batch_get_tuning")
    return t.items, t.radix_bits, t.small_cap


def qsd_batch_workspace(batch):
    n = ctypes.c_size_t()
    _check(load().qsd_batch_workspace(batch, ctypes.byref(n)), "qsd_batch_workspace")
    return n.value


def qsd_batch_workspace_max(batch):
    n = ctypes.c_size_t()
    _check(load().qsd_batch_workspace_max(batch, ctypes.byref(n)), "qsd_batch_workspace_max")
    return n.value


def _ios(ios):
    """ios: sequence of (in_crd ptrs, in_val ptr, out_crd ptrs, out_val ptr)."""
    arr = (qsd_batch_io * max(len(ios), 1))()
    for i, (ic, iv, oc, ov) in enumerate(ios):
        for m, p in enumerate(ic):
            arr[i].in_crd[m] = p
        for m, p in enumerate(oc):
            arr[i].out_crd[m] = p
        arr[i].in_val = iv
        arr[i].out_val = ov
    return arr


def qsd_batch_bind(batch, ios, ws, ws_bytes, stream):
    _check(load().qsd_batch_bind(batch, _ios(ios), ws, int(ws_bytes), stream), "qsd_batch_bind")


def qsd_batch_transpose(batch, ws, ws_bytes, stream):
    _check(load().qsd_batch_transpose(batch, ws, int(ws_bytes), stream), "qsd_batch_transpose")


def qsd_batch_tune(batch, ios, ws, ws_bytes, stream, reps=3):
    """Returns ((items, radix_bits, small_cap), best_ms)."""
    t = qsd_tuning()
    ms = ctypes.c_float()
    _check(load().qsd_batch_tune(batch, _ios(ios), ws, int(ws_bytes), stream, int(reps), ctypes.byref(t),
                                 ctypes.byref(ms)), "qsd_batch_tune")
    return (t.items, t.radix_bits, t.small_cap), ms.value


def qsd_batch_tune_key(batch):
    buf = ctypes.create_string_buffer(128)
    _check(load().qsd_batch_tune_key(batch, buf, len(buf)), "qsd_batch_tune_key")
    return buf.value.decode()


def qsd_batch_tune_cached(batch, ios, ws, ws_bytes, stream, cache_path, reps=3):
    """Returns ((items, radix_bits, small_cap), best_ms, from_cache)."""
    t = qsd_tuning()
    ms = ctypes.c_float()
    hit = ctypes.c_int32()
    _check(load().qsd_batch_tune_cached(batch, _ios(ios), ws, int(ws_bytes), stream, int(reps),
                                        str(cache_path).encode(), ctypes.byref(t), ctypes.byref(ms),
                                        ctypes.byref(hit)), "qsd_batch_tune_cached")
    return (t.items, t.radix_bits, t.small_cap), ms.value, bool(hit.value)


def qsd_batch_graph(batch, ws, ws_bytes):
    h = _VP()
    _check(load().qsd_batch_graph(batch, ws, int(ws_bytes), ctypes.byref(h)), "qsd_batch_graph")
    return h.value


def qsd_graph_launch(graph, stream):
    _check(load().qsd_graph_launch(graph, stream), "qsd_graph_launch")


def qsd_graph_destroy(graph):
    load().qsd_graph_destroy(graph)


NFEAT, NCAND, MLP_NPARAM, FEAT_COUNTS = 40, 6, 7174, 3 * (MAX_ORDER + 4)
# the selector's candidates: (name, schedule for qsd_plan, extra plan flags)
CANDIDATES = (("minimal", "minimal", 0), ("minimal-buckets", "minimal", QSD_KEEP_BUCKETS), ("topk1", "topk1", 0),
              ("topk2", "topk2", 0), ("topk3", "topk3", 0), ("lsd", "lsd", 0))
CAND_NAMES = tuple(c[0] for c in CANDIDATES)


def qsd_candidate(c):
    """(schedule code, extra plan flags) of candidate c."""
    sc = ctypes.c_int()
    fl = ctypes.c_uint32()
    _check(load().qsd_candidate(int(c), ctypes.byref(sc), ctypes.byref(fl)), "qsd_candidate")
    return sc.value, fl.value


def qsd_candidate_terms(desc):
    """[(valid, global digit passes, bucketed key bits)] of every candidate of a request."""
    d, _keep = _desc(*desc)
    v, gp, sb = (ctypes.c_int32 * NCAND)(), (ctypes.c_int32 * NCAND)(), (ctypes.c_int32 * NCAND)()
    _check(load().qsd_candidate_terms(ctypes.byref(d), v, gp, sb), "qsd_candidate_terms")
    return [(bool(v[c]), gp[c], sb[c]) for c in range(NCAND)]


def qsd_candidates_valid(desc):
    return [t[0] for t in qsd_candidate_terms(desc)]


def qsd_select_workspace():
    n = ctypes.c_size_t()
    _check(load().qsd_select_workspace(ctypes.byref(n)), "qsd_select_workspace")
    return n.value


def qsd_feature_counts(desc, in_crd, ws, ws_bytes, stream):
    """desc: (order, nnz, extents, crd_type, val_type, in_order, out_order).
    Returns (counts list of FEAT_COUNTS ints, S, pairs)."""
    d, _keep = _desc(*desc)
    out = (ctypes.c_uint32 * FEAT_COUNTS)()
    S, P = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().qsd_feature_counts(ctypes.byref(d), _ptrs(in_crd), ws, int(ws_bytes), stream, out,
                                     ctypes.byref(S), ctypes.byref(P)), "qsd_feature_counts")
    return list(out), S.value, P.value


def qsd_features(desc, in_crd, ws, ws_bytes, stream):
    d, _keep = _desc(*desc)
    out = (ctypes.c_float * NFEAT)()
    _check(load().qsd_features(ctypes.byref(d), _ptrs(in_crd), ws, int(ws_bytes), stream, out), "qsd_features")
    return list(out)


def qsd_mlp_init(seed):
    out = (ctypes.c_float * MLP_NPARAM)()
    _check(load().qsd_mlp_init(ctypes.c_uint64(int(seed)), out), "qsd_mlp_init")
    return list(out)


def qsd_mlp_forward(params, x, n, h1, h2, y, stream):
    _check(load().qsd_mlp_forward(params, x, int(n), h1, h2, y, stream), "qsd_mlp_forward")


def qsd_mlp_backward_workspace(n):
    b = ctypes.c_size_t()
    _check(load().qsd_mlp_backward_workspace(int(n), ctypes.byref(b)), "qsd_mlp_backward_workspace")
    return b.value


def qsd_mlp_backward(params, x, h1, h2, y, t, n, grad, loss, ws, ws_bytes, stream):
    _check(load().qsd_mlp_backward(params, x, h1, h2, y, t, int(n), grad, loss, ws, int(ws_bytes), stream),
           "qsd_mlp_backward")


def qsd_mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, stream):
    _check(load().qsd_mlp_adam(params, grad, m, v, int(step), lr, beta1, beta2, eps, stream), "qsd_mlp_adam")


def qsd_mlp_train_workspace(n, batch):
    b = ctypes.c_size_t()
    _check(load().qsd_mlp_train_workspace(int(n), int(batch), ctypes.byref(b)), "qsd_mlp_train_workspace")
    return b.value


def qsd_mlp_train(params, x, t, n, epochs, batch, lr, seed, ws, ws_bytes, stream):
    loss = ctypes.c_float()
    _check(load().qsd_mlp_train(params, x, t, int(n), int(epochs), int(batch), float(lr),
                                ctypes.c_uint64(int(seed)), ws, int(ws_bytes), stream, ctypes.byref(loss)),
           "qsd_mlp_train")
    return loss.value


def qsd_model_create(params, margin, min_nnz=0):
    arr = (ctypes.c_float * MLP_NPARAM)(*[float(x) for x in params])
    h = _VP()
    _check(load().qsd_model_create(arr, float(margin), int(min_nnz), ctypes.byref(h)), "qsd_model_create")
    return h.value


def qsd_model_load(path):
    h = _VP()
    _check(load().qsd_model_load(os.fsencode(path), ctypes.byref(h)), "qsd_model_load")
    return h.value


def qsd_model_destroy(model):
    load().qsd_model_destroy(model)


def qsd_select(model, desc, in_crd, ws, ws_bytes, stream):
    """Returns (chosen candidate, predicted log2 ms of every candidate)."""
    d, _keep = _desc(*desc)
    ch = ctypes.c_int32()
    pred = (ctypes.c_float * NCAND)()
    _check(load().qsd_select(model, ctypes.byref(d), _ptrs(in_crd), ws, int(ws_bytes), stream, ctypes.byref(ch),
                             pred), "qsd_select")
    return ch.value, list(pred)


def qsd_plan_auto(model, desc, in_crd, ws, ws_bytes, stream):
    """Returns (plan handle, chosen candidate)."""
    d, _keep = _desc(*desc)
    h = _VP()
    ch = ctypes.c_int32()
    _check(load().qsd_plan_auto(model, ctypes.byref(d), _ptrs(in_crd), ws, int(ws_bytes), stream,
                                ctypes.byref(h), ctypes.byref(ch)), "qsd_plan_auto")
    return h.value, ch.value


def write_model_file(path, params, margin, min_nnz=0):
    """The selector weights file read by qsd_model_load."""
    import struct
    with open(path, "wb") as f:
        f.write(b"QSDMLP2\0")
        f.write(struct.pack("<ifq", MLP_NPARAM, float(margin), int(min_nnz)))
        f.write(struct.pack(f"<{MLP_NPARAM}f", *[float(x) for x in params]))


def qsd_status_str(code):
    return load().qsd_status_str(int(code)).decode()


# ---------------------------------------------------------------- torch convenience layer

class Plan:
    """A plan plus the torch plumbing to call it on CUDA (HIP) tensors."""

    def __init__(self, extents, in_order, out_order, nnz, crd_dtype="int32", val_dtype="float64",
                 sched="minimal", flags=0, model=None, crd=None):
        """sched="auto" with a selector `model` (qsd_model_load) and the input coordinates
        `crd` (device tensors) chooses the schedule with qsd_plan_auto."""
        import torch
        self.torch = torch
        self.r = len(extents)
        self.extents = tuple(int(x) for x in extents)
        self.in_order = tuple(int(x) for x in in_order)
        self.out_order = tuple(int(x) for x in out_order)
        self.nnz = int(nnz)
        self.crd_dtype = getattr(torch, str(crd_dtype).replace("torch.", ""))
        self.val_dtype = getattr(torch, str(val_dtype).replace("torch.", ""))
        ct = QSD_I64 if self.crd_dtype == torch.int64 else QSD_I32
        vt = QSD_F64 if self.val_dtype == torch.float64 else QSD_F32
        self.chosen = None
        if sched == "auto" and model is not None:
            sws = torch.empty(qsd_select_workspace(), dtype=torch.uint8, device=crd[0].device)
            self.handle, self.chosen = qsd_plan_auto(
                model, (self.r, self.nnz, self.extents, ct, vt, self.in_order, self.out_order),
                [c.data_ptr() for c in crd], sws.data_ptr(), sws.numel(),
                torch.cuda.current_stream(crd[0].device).cuda_stream)
        else:
            self.handle = qsd_plan(self.r, self.nnz, self.extents, ct, vt, self.in_order, self.out_order,
                                   sched, flags)
        self.ws_bytes = qsd_plan_workspace(self.handle)
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                qsd_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def describe(self):
        return qsd_plan_describe(self.handle)

    def workspace(self, device="cuda"):
        if self._ws is None or self._ws.numel() < self.ws_bytes:
            self._ws = self.torch.empty(max(self.ws_bytes, 1), dtype=self.torch.uint8, device=device)
        return self._ws

    def transpose(self, crd, val, out_crd=None, out_val=None, stream=None, nnz=None, ws=None):
        """ws: optional uint8 device tensor of at least ws_bytes (shared between plans that
        run one after the other on one stream)."""
        torch = self.torch
        n = int(val.shape[0]) if nnz is None else int(nnz)
        dev = val.device
        if out_crd is None:
            out_crd = [torch.empty_like(c) for c in crd]
        if out_val is None:
            out_val = torch.empty_like(val)
        if ws is None:
            ws = self.workspace(dev)
        elif ws.numel() < self.ws_bytes:
            raise ValueError("workspace tensor smaller than the plan needs")
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        qsd_transpose(self.handle, n, [c.data_ptr() for c in crd], val.data_ptr(),
                      [c.data_ptr() for c in out_crd], out_val.data_ptr(), ws.data_ptr(), self.ws_bytes,
                      s.cuda_stream)
        self._last_ws = ws
        return out_crd, out_val

    def device_status(self, stream=None):
        """Status bits of the calls since the last read, on the workspace the last call used."""
        s = stream if stream is not None else self.torch.cuda.current_stream()
        ws = getattr(self, "_last_ws", None)
        if ws is None:
            return 0  # nothing has run
        return qsd_device_status(ws.data_ptr(), s.cuda_stream)

    def transpose_csf(self, in_pos, in_crd, in_val, stream=None):
        """CSF (levels in in_order) -> CSF (levels in out_order): returns (pos list, crd list,
        values, fiber counts as a host list)."""
        torch = self.torch
        n = int(in_val.shape[0])
        dev = in_val.device
        pt = torch.int64 if self.crd_dtype == torch.int64 else torch.int32
        pos = [torch.empty(2 if d == 0 else max(n, 1) + 1, dtype=pt, device=dev) for d in range(self.r)]
        crd = [torch.empty(max(n, 1), dtype=self.crd_dtype, device=dev) for _ in range(self.r)]
        val = torch.empty_like(in_val)
        fc = torch.empty(self.r + 1, dtype=torch.int64, device=dev)
        wsb = qsd_csf_transpose_workspace(self.handle)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        qsd_csf_transpose(self.handle, n, [p.data_ptr() for p in in_pos], [c.data_ptr() for c in in_crd],
                          in_val.data_ptr(), [p.data_ptr() for p in pos], [c.data_ptr() for c in crd],
                          val.data_ptr(), fc.data_ptr(), ws.data_ptr(), wsb, s.cuda_stream)
        self._last_ws = ws
        counts = fc.cpu().tolist()
        return ([pos[d][:counts[d] + 1] for d in range(self.r)], [crd[d][:counts[d + 1]] for d in range(self.r)],
                val, counts)

    def pack_csf(self, sorted_crd, nnz=None, stream=None):
        """CSF of a tensor sorted under out_order: returns (pos list, crd list, fiber counts)."""
        torch = self.torch
        n = int(sorted_crd[0].shape[0]) if nnz is None else int(nnz)
        dev = sorted_crd[0].device
        pt = torch.int64 if self.crd_dtype == torch.int64 else torch.int32
        pos = [torch.empty(2 if d == 0 else n + 1, dtype=pt, device=dev) for d in range(self.r)]
        crd = [torch.empty(max(n, 1), dtype=self.crd_dtype, device=dev) for _ in range(self.r)]
        fc = torch.empty(self.r + 1, dtype=torch.int64, device=dev)
        wsb = qsd_csf_workspace(self.handle)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        qsd_pack_csf(self.handle, n, [c.data_ptr() for c in sorted_crd], [p.data_ptr() for p in pos],
                     [c.data_ptr() for c in crd], fc.data_ptr(), ws.data_ptr(), wsb, s.cuda_stream)
        s.synchronize()
        counts = [int(x) for x in fc.cpu()]
        pos = [pos[d][: counts[d] + 1] for d in range(self.r)]
        crd = [crd[d][: counts[d + 1]] for d in range(self.r)]
        return pos, crd, counts


class Batch:
    """Many transpositions in a few launches (optionally one HIP graph), on torch tensors.

    tensors: list of dicts with keys crd (list of r device tensors), val, extents,
    in_order, out_order.  Output tensors are allocated once and reused by every call."""

    def __init__(self, tensors, device="cuda"):
        import torch
        self.torch = torch
        self.tensors = tensors
        ct = QSD_I64 if tensors and tensors[0]["crd"][0].dtype == torch.int64 else QSD_I32
        vt = QSD_F64 if tensors and tensors[0]["val"].dtype == torch.float64 else QSD_F32
        descs = [(len(t["crd"]), int(t["val"].shape[0]), t["extents"], ct, vt, t["in_order"], t["out_order"])
                 for t in tensors]
        self.handle = qsd_batch_plan(descs)
        self.out_crd = [[torch.empty_like(c) for c in t["crd"]] for t in tensors]
        self.out_val = [torch.empty_like(t["val"]) for t in tensors]
        self.ws_bytes = qsd_batch_workspace_max(self.handle)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.graph = None
        self.bind()

    def __del__(self):
        g = getattr(self, "graph", None)
        if g:
            try:
                qsd_graph_destroy(g)
            except Exception:
                pass
        h = getattr(self, "handle", None)
        if h:
            try:
                qsd_batch_destroy(h)
            except Exception:
                pass
            self.handle = None

    def _io(self):
        return [([c.data_ptr() for c in t["crd"]], t["val"].data_ptr(), [c.data_ptr() for c in oc], ov.data_ptr())
                for t, oc, ov in zip(self.tensors, self.out_crd, self.out_val)]

    def _stream(self, stream):
        return (stream if stream is not None else self.torch.cuda.current_stream()).cuda_stream

    def bind(self, stream=None):
        qsd_batch_bind(self.handle, self._io(), self.ws.data_ptr(), self.ws_bytes, self._stream(stream))

    def set_tuning(self, items, radix_bits, small_cap, stream=None):
        qsd_batch_set_tuning(self.handle, items, radix_bits, small_cap)
        self.bind(stream)

    def tuning(self):
        return qsd_batch_get_tuning(self.handle)

    def tune(self, reps=3, stream=None, cache=None):
        """The autotuner; with `cache` (a file path) a cached tuning for this batch's key is
        applied without timing, and a new result is appended.  Returns (tuning, ms) without a
        cache, (tuning, ms, from_cache) with one."""
        if cache is not None:
            return qsd_batch_tune_cached(self.handle, self._io(), self.ws.data_ptr(), self.ws_bytes,
                                         self._stream(stream), cache, reps)
        return qsd_batch_tune(self.handle, self._io(), self.ws.data_ptr(), self.ws_bytes, self._stream(stream), reps)

    def tune_key(self):
        return qsd_batch_tune_key(self.handle)

    def transpose(self, stream=None):
        qsd_batch_transpose(self.handle, self.ws.data_ptr(), self.ws_bytes, self._stream(stream))
        return self.out_crd, self.out_val

    def capture(self):
        if self.graph:
            qsd_graph_destroy(self.graph)
        self.graph = qsd_batch_graph(self.handle, self.ws.data_ptr(), self.ws_bytes)

    def replay(self, stream=None):
        qsd_graph_launch(self.graph, self._stream(stream))
        return self.out_crd, self.out_val

    def device_status(self, stream=None):
        return qsd_device_status(self.ws.data_ptr(), self._stream(stream))
