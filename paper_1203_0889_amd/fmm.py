"""Python binding of the C ABI in include/fmm.h (ctypes; argument marshalling only).

Every step of the method runs in the HIP library libfmm_mi355x.so; torch is
used for device memory and the current HIP stream.  There is no fallback: if
the library is missing, loading fails with an error.

    plan = Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed")
    plan.build_tree(pos, q)          # pos (N, 3) float64 cuda, q (N,) float64 cuda
    plan.upward()
    out = plan.evaluate()            # dict: phi, field, force, energy
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm_mi355x.so")

FMM_OK = 0
STATUS = {0: "FMM_OK", -1: "FMM_ERR_INVALID_ARG", -2: "FMM_ERR_STATE", -3: "FMM_ERR_OOM",
          -4: "FMM_ERR_DEVICE", -5: "FMM_ERR_CAPACITY", -6: "FMM_ERR_UNSUPPORTED"}
PREC = {"fp64": 0, "mixed": 1}
FLAG_USER_BOX = 1
FLAG_KEEP_TOPOLOGY = 2
FLAG_TRACE = 4
FLAG_DETERMINISTIC = 8
FLAG_INCREMENTAL = 16
FLAG_COST_REUSE = 32
FLAG_MUTUAL_M2L = 64
FLAG_MUTUAL_P2P = 128
FLAG_MUTUAL = FLAG_MUTUAL_M2L | FLAG_MUTUAL_P2P
MUTUAL = {False: 0, None: 0, True: FLAG_MUTUAL, "both": FLAG_MUTUAL, "m2l": FLAG_MUTUAL_M2L, "p2p": FLAG_MUTUAL_P2P}

# every symbol include/fmm.h declares
EXPORTS = ("fmm_default_params", "fmm_create", "fmm_destroy", "fmm_build_tree", "fmm_upward", "fmm_evaluate",
           "fmm_backward", "fmm_sync", "fmm_get_counts", "fmm_copy_tree", "fmm_copy_lists", "fmm_get_tuning",
           "fmm_set_tuning", "fmm_get_stage_times", "fmm_status_string", "fmm_last_error", "fmm_graph_capture",
           "fmm_graph_launch", "fmm_autotune", "fmm_get_trace", "fmm_get_queue_info", "fmm_evaluate_noalloc",
           "fmm_graph_capture_step", "fmm_get_build_info")


class fmm_params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("ncrit", ctypes.c_int32), ("theta_num", ctypes.c_int32),
                ("theta_den", ctypes.c_int32), ("max_level", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("box_min", ctypes.c_double * 3), ("box_side", ctypes.c_double)]


class fmm_tuning(ctypes.Structure):
    _fields_ = [("m2l_task_entries", ctypes.c_int32), ("grid_per_cu", ctypes.c_int32), ("p2p_per_cu", ctypes.c_int32),
                ("early_p2p_per_cu", ctypes.c_int32)]


class fmm_task_record(ctypes.Structure):
    _fields_ = [("start", ctypes.c_uint64), ("end", ctypes.c_uint64), ("kind", ctypes.c_int32),
                ("task", ctypes.c_int32), ("kernel", ctypes.c_int32), ("hw_id", ctypes.c_uint32),
                ("xcc", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


# the same layout as a numpy record (ticks of the 100 MHz device clock)
TASK_DTYPE = np.dtype([("start", "<u8"), ("end", "<u8"), ("kind", "<i4"), ("task", "<i4"), ("kernel", "<i4"),
                       ("hw_id", "<u4"), ("xcc", "<u4"), ("reserved", "<u4")])


class FMMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None


def load_library():
    """Load libfmm_mi355x.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library %s is missing: build it first "
                          "(python paper_1203_0889_amd/build.py)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    lib.fmm_default_params.argtypes = [P(fmm_params)]
    lib.fmm_create.argtypes = [P(fmm_params), ctypes.c_int, vp, P(vp)]
    lib.fmm_destroy.argtypes = [vp]
    lib.fmm_build_tree.argtypes = [vp, i32, P(i64), vp, vp]
    lib.fmm_upward.argtypes = [vp]
    lib.fmm_evaluate.argtypes = [vp, vp, vp, vp, vp]
    lib.fmm_evaluate_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.fmm_backward.argtypes = [vp, vp, vp, vp]
    lib.fmm_sync.argtypes = [vp]
    lib.fmm_graph_capture.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.fmm_graph_capture_step.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.fmm_graph_launch.argtypes = [vp]
    lib.fmm_get_build_info.argtypes = [vp, P(i64), P(i64)]
    lib.fmm_autotune.argtypes = [vp, i32, P(fmm_tuning), P(ctypes.c_double)]
    lib.fmm_get_counts.argtypes = [vp, P(i64), P(i64), P(i64), P(i64)]
    lib.fmm_get_queue_info.argtypes = [vp, P(i64), P(i64), P(i64), P(i64), P(i64)]
    lib.fmm_copy_tree.argtypes = [vp, vp, vp, vp]
    lib.fmm_copy_lists.argtypes = [vp, vp, vp, vp, vp]
    lib.fmm_get_tuning.argtypes = [vp, P(fmm_tuning)]
    lib.fmm_set_tuning.argtypes = [vp, P(fmm_tuning)]
    lib.fmm_get_stage_times.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_char_p)]
    lib.fmm_get_trace.argtypes = [vp, vp, i64, P(i64)]
    lib.fmm_status_string.argtypes = [ctypes.c_int]
    lib.fmm_status_string.restype = ctypes.c_char_p
    lib.fmm_last_error.argtypes = [vp]
    lib.fmm_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("fmm_status_string", "fmm_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_dev(t, name, dtype=torch.float64, shape_tail=(), shape=None, device=None):
    """A device tensor the library reads or writes: the kernels index it as a
    contiguous FP64 array of the given shape, so anything else is refused
    here, before a pointer reaches the library."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor on the GPU" % (name, dtype))
    if device is not None and t.device.index != device:
        raise ValueError("%s must be on cuda:%d, the plan's device" % (name, device))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, not %s" % (name, tuple(shape), tuple(t.shape)))
    if shape_tail and tuple(t.shape[1:]) != shape_tail:
        raise ValueError("%s must have shape (N, %s)" % (name, ", ".join(map(str, shape_tail))))


class Plan:
    """One FMM plan: owns the tree, lists and expansions on one device/stream."""

    def __init__(self, p=8, ncrit=64, theta=(1, 2), max_level=21, precision="mixed", device=None, stream=None,
                 box=None, keep_topology=False, trace=False, deterministic=False, incremental=False,
                 cost_reuse=False, mutual=False):
        self._lib = load_library()
        prm = fmm_params()
        self._lib.fmm_default_params(ctypes.byref(prm))
        prm.p, prm.ncrit = int(p), int(ncrit)
        prm.theta_num, prm.theta_den = int(theta[0]), int(theta[1])
        prm.max_level = int(max_level)
        prm.precision = PREC[precision]
        if box is not None:
            prm.flags |= FLAG_USER_BOX
            prm.box_min[0], prm.box_min[1], prm.box_min[2] = map(float, box[:3])
            prm.box_side = float(box[3])
        if keep_topology:
            prm.flags |= FLAG_KEEP_TOPOLOGY
        if trace:
            prm.flags |= FLAG_TRACE
        if deterministic:
            prm.flags |= FLAG_DETERMINISTIC
        if incremental:
            prm.flags |= FLAG_INCREMENTAL
        if cost_reuse:
            prm.flags |= FLAG_COST_REUSE
        if mutual not in MUTUAL:
            raise ValueError("mutual must be False, True, 'both', 'm2l' or 'p2p'")
        prm.flags |= MUTUAL[mutual]   # FP64: the mutual interaction for M2L, P2P or both
        self.params = prm
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self._lib.fmm_create(ctypes.byref(prm), self.device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != FMM_OK:
            raise FMMError(st, "fmm_create failed")
        self._h = h
        self.n = 0
        self.n_inst = 0
        self._keep = None

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.fmm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, *args):
        st = fn(self._h, *args)
        if st != FMM_OK:
            raise FMMError(st, self._lib.fmm_last_error(self._h).decode())

    # ---- the four calls of the method
    def build_tree(self, pos, q, offsets=None):
        """Keys, sort, octree and interaction lists.  offsets (host ints,
        n_inst + 1) batches independent instances."""
        _check_dev(pos, "pos", shape_tail=(3,), device=self.device)
        _check_dev(q, "q", device=self.device)
        n = pos.shape[0]
        if q.shape != (n,):
            raise ValueError("q must have shape (N,)")
        if offsets is None:
            offsets = [0, n]
        offs = (ctypes.c_int64 * len(offsets))(*[int(o) for o in offsets])
        self._call(self._lib.fmm_build_tree, ctypes.c_int32(len(offsets) - 1), offs, _ptr(pos), _ptr(q))
        self.n = n
        self.n_inst = len(offsets) - 1
        self._keep = (pos, q)

    def upward(self):
        self._call(self._lib.fmm_upward)

    def evaluate(self, phi=True, field=True, force=True, energy=True):
        dev = torch.device("cuda", self.device)
        out = {}
        n = self.n
        out["phi"] = torch.empty(n, dtype=torch.float64, device=dev) if phi else None
        out["field"] = torch.empty((n, 3), dtype=torch.float64, device=dev) if field else None
        out["force"] = torch.empty((n, 3), dtype=torch.float64, device=dev) if force else None
        out["energy"] = torch.empty(self.n_inst, dtype=torch.float64, device=dev) if energy else None
        self._call(self._lib.fmm_evaluate, _ptr(out["phi"]), _ptr(out["field"]), _ptr(out["force"]),
                   _ptr(out["energy"]))
        return out

    def _check_outputs(self, **named):
        """Shapes the library writes: phi (N,), field and force (N, 3),
        energy (n_inst,), grad_pos (N, 3), grad_q (N,), grad_energy (n_inst,)."""
        shapes = {"phi": (self.n,), "field": (self.n, 3), "force": (self.n, 3), "energy": (self.n_inst,),
                  "grad_energy": (self.n_inst,), "grad_pos": (self.n, 3), "grad_q": (self.n,)}
        for name, t in named.items():
            if t is not None:
                _check_dev(t, name, shape=shapes[name], device=self.device)

    def evaluate_into(self, phi=None, field=None, force=None, energy=None):
        self._check_outputs(phi=phi, field=field, force=force, energy=energy)
        self._call(self._lib.fmm_evaluate, _ptr(phi), _ptr(field), _ptr(force), _ptr(energy))

    def evaluate_noalloc_into(self, phi=None, field=None, force=None, energy=None):
        """fmm_evaluate_noalloc: the evaluation into caller-owned outputs with
        no device allocation (the plan's workspaces must already be sized)."""
        self._check_outputs(phi=phi, field=field, force=force, energy=energy)
        self._call(self._lib.fmm_evaluate_noalloc, _ptr(phi), _ptr(field), _ptr(force), _ptr(energy))

    def backward(self, grad_energy, want_pos=True, want_q=True):
        """Gradient of sum_k grad_energy[k] E_k (the FMM's energies) with
        respect to positions and charges: (grad_pos (N, 3), grad_q (N,))."""
        dev = torch.device("cuda", self.device)
        self._check_outputs(grad_energy=grad_energy)
        gp = torch.empty((self.n, 3), dtype=torch.float64, device=dev) if want_pos else None
        gq = torch.empty(self.n, dtype=torch.float64, device=dev) if want_q else None
        self._call(self._lib.fmm_backward, _ptr(grad_energy), _ptr(gp), _ptr(gq))
        return gp, gq

    # ---- HIP graph of upward + evaluate (+ backward)
    def graph_capture(self, phi=None, field=None, force=None, energy=None, grad_energy=None, grad_pos=None,
                      grad_q=None):
        """Capture upward + evaluate (+ backward when grad_energy is given)
        into a HIP graph writing into the given tensors."""
        self._check_outputs(phi=phi, field=field, force=force, energy=energy, grad_energy=grad_energy,
                            grad_pos=grad_pos, grad_q=grad_q)
        self._graph_refs = (phi, field, force, energy, grad_energy, grad_pos, grad_q)
        self._call(self._lib.fmm_graph_capture, _ptr(phi), _ptr(field), _ptr(force), _ptr(energy), _ptr(grad_energy),
                   _ptr(grad_pos), _ptr(grad_q))

    def graph_capture_step(self, pos, q, phi=None, field=None, force=None, energy=None):
        """Capture a whole time step (frozen-topology rebuild from pos / q,
        upward, evaluate) into a HIP graph; every replay reads pos and q
        again, so write the next step's positions into the same tensors."""
        _check_dev(pos, "pos", shape=(self.n, 3), device=self.device)
        _check_dev(q, "q", shape=(self.n,), device=self.device)
        self._check_outputs(phi=phi, field=field, force=force, energy=energy)
        self._graph_refs = (pos, q, phi, field, force, energy)
        self._call(self._lib.fmm_graph_capture_step, _ptr(pos), _ptr(q), _ptr(phi), _ptr(field), _ptr(force),
                   _ptr(energy))

    def graph_launch(self):
        self._call(self._lib.fmm_graph_launch)

    # ---- introspection
    def sync(self):
        self._call(self._lib.fmm_sync)

    def counts(self):
        v = [ctypes.c_int64() for _ in range(4)]
        self._call(self._lib.fmm_get_counts, *[ctypes.byref(x) for x in v])
        return dict(zip(("ncell", "nleaf", "nm2l", "np2p"), (x.value for x in v)))

    def build_info(self):
        """fmm_build_tree calls so far: built from scratch / on a kept topology."""
        v = [ctypes.c_int64() for _ in range(2)]
        self._call(self._lib.fmm_get_build_info, *[ctypes.byref(x) for x in v])
        return {"full": v[0].value, "kept": v[1].value}

    def queue_info(self):
        """Class-table and work-queue sizes of the last build (the FP64 path
        reports its class tables; zeros where M2L runs per pair: p > 12 or
        mutual)."""
        v = [ctypes.c_int64() for _ in range(5)]
        self._call(self._lib.fmm_get_queue_info, *[ctypes.byref(x) for x in v])
        return dict(zip(("ntarget", "ngroup", "ntask", "nclass", "nextra"), (x.value for x in v)))

    def copy_tree(self):
        import numpy as np
        c = self.counts()
        keys = np.zeros(self.n, dtype=np.uint64)
        perm = np.zeros(self.n, dtype=np.int64)
        cells = np.zeros((c["ncell"], 10), dtype=np.int64)
        self._call(self._lib.fmm_copy_tree, ctypes.c_void_p(keys.ctypes.data), ctypes.c_void_p(perm.ctypes.data),
                   ctypes.c_void_p(cells.ctypes.data))
        return keys, perm, cells

    def copy_lists(self):
        import numpy as np
        c = self.counts()
        mp = np.zeros(c["ncell"] + 1, dtype=np.int64)
        pp = np.zeros(c["ncell"] + 1, dtype=np.int64)
        ms = np.zeros(max(c["nm2l"], 1), dtype=np.int32)
        ps = np.zeros(max(c["np2p"], 1), dtype=np.int32)
        self._call(self._lib.fmm_copy_lists, ctypes.c_void_p(mp.ctypes.data), ctypes.c_void_p(ms.ctypes.data),
                   ctypes.c_void_p(pp.ctypes.data), ctypes.c_void_p(ps.ctypes.data))
        return mp, ms[:c["nm2l"]], pp, ps[:c["np2p"]]

    def stage_times(self):
        t = (ctypes.c_double * 16)()
        names = (ctypes.c_char_p * 16)()
        self._call(self._lib.fmm_get_stage_times, t, names)
        return {names[i].decode(): t[i] for i in range(16) if names[i] and names[i].decode()}

    def trace(self):
        """Task records of the last traced evaluate (numpy array of TASK_DTYPE)."""
        n = ctypes.c_int64()
        self._call(self._lib.fmm_get_trace, None, 0, ctypes.byref(n))
        out = np.zeros(n.value, dtype=TASK_DTYPE)
        if n.value:
            self._call(self._lib.fmm_get_trace, ctypes.c_void_p(out.ctypes.data), n.value, ctypes.byref(n))
        return out[:n.value]

    def get_tuning(self):
        t = fmm_tuning()
        self._call(self._lib.fmm_get_tuning, ctypes.byref(t))
        return {f: getattr(t, f) for f, _ in fmm_tuning._fields_}

    def autotune(self, repeats=3):
        """Sweep the work-queue settings on the current tree and multipoles
        (after upward); keeps the fastest.  Returns (tuning dict, queue ms)."""
        t = fmm_tuning()
        ms = ctypes.c_double()
        self._call(self._lib.fmm_autotune, ctypes.c_int32(int(repeats)), ctypes.byref(t), ctypes.byref(ms))
        return {f: getattr(t, f) for f, _ in fmm_tuning._fields_}, ms.value

    def set_tuning(self, **kw):
        t = fmm_tuning()
        self._call(self._lib.fmm_get_tuning, ctypes.byref(t))
        for k, v in kw.items():
            setattr(t, k, int(v))
        self._call(self._lib.fmm_set_tuning, ctypes.byref(t))


def evaluate(pos, q, p=8, ncrit=64, theta=(1, 2), precision="mixed", **kw):
    """One-shot FMM: returns (phi, field) in input order."""
    plan = Plan(p=p, ncrit=ncrit, theta=theta, precision=precision, **kw)
    plan.build_tree(pos, q)
    plan.upward()
    out = plan.evaluate(force=False, energy=False)
    return out["phi"], out["field"]
