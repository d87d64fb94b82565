"""ctypes binding of libqwalk.so (the C ABI in include/qwalk.h).

Argument marshalling only: every step of the walk runs in the library's HIP
kernels.  The library is loaded after torch so that both share torch's HIP
runtime (same SONAME); if it is missing, loading fails loudly -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqwalk.so")

QW_OK, QW_EINVAL, QW_EGRAPH, QW_EUNSUPPORTED, QW_ENOMEM, QW_EDEVICE, QW_ESTATE = range(7)
ERRORS = {1: "QW_EINVAL", 2: "QW_EGRAPH", 3: "QW_EUNSUPPORTED", 4: "QW_ENOMEM", 5: "QW_EDEVICE",
          6: "QW_ESTATE"}
QW_COINED, QW_CTQW, QW_STAGGERED = 0, 1, 2
QW_REFLECTION, QW_HAMILTONIAN = 0, 1
QW_GROVER, QW_HADAMARD, QW_FOURIER, QW_MATRIX, QW_SZEGEDY = 0, 1, 2, 3, 4
QW_FLIPFLOP, QW_PERSISTENT = 0, 1
QW_C64, QW_C128 = 0, 1
QW_BATCH_GATHER, QW_BATCH_LDS = 0, 1
QW_STREAM_DIRECT, QW_STREAM_RING = 0, 1
QW_LAYOUT_AUTO, QW_LAYOUT_CSR, QW_LAYOUT_STRUCTURED, QW_LAYOUT_DENSE = 0, 1, 2, 3
STRUCTURES = {0: "general", 1: "cycle", 2: "torus", 3: "hypercube", 4: "small", 5: "ell", 6: "dense",
              7: "stag_lattice"}

EXPORTS = ["qw_plan_create", "qw_plan_destroy", "qw_plan_get_info", "qw_plan_upload", "qw_evolve",
           "qw_probabilities", "qw_copy_to_host", "qw_small_many_desc_bytes", "qw_small_many",
           "qw_taylor_order", "qw_taylor_plan", "qw_taylor_tail_bound",
           "qw_last_error", "qw_version",
           "qw_batch_create", "qw_batch_destroy", "qw_batch_device_bytes", "qw_batch_bind",
           "qw_batch_set_slot", "qw_batch_clear_slot", "qw_batch_commit", "qw_batch_run",
           "qw_batch_remaining", "qw_batch_launches", "qw_batch_readout", "qw_batch_set_schedule",
           "qw_batch_autotune", "qw_batch_set_replay", "qw_batch_launch_plan", "qw_batch_set_stage_kernel",
           "qw_batch_get_schedule", "qw_plan_stream_sizes", "qw_plan_upload_streamed", "qw_evolve_static"]


class QwCsr(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32))]


class QwTessellation(C.Structure):
    _fields_ = [("n_polygons", C.c_int64), ("poly_ptr", C.POINTER(C.c_int64)), ("poly_vert", C.POINTER(C.c_int32)),
                ("amp", C.POINTER(C.c_double)), ("form", C.c_int32), ("theta", C.c_double)]


class QwWalkDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("coin", C.c_int32), ("dtype", C.c_int32), ("layout", C.c_int32),
                ("gamma", C.c_double), ("dt", C.c_double), ("taylor_order", C.c_int32),
                ("trunc_tol", C.c_double), ("horizon_steps", C.c_int64),
                ("marked", C.POINTER(C.c_int32)), ("n_marked", C.c_int64), ("columns", C.c_int32),
                ("shift", C.c_int32), ("coin_dim", C.c_int32), ("coin_matrix", C.POINTER(C.c_double)),
                ("transition", C.POINTER(C.c_double)), ("n_tessellations", C.c_int32),
                ("tessellations", C.POINTER(QwTessellation))]


class QwPlanInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_arcs", C.c_int64), ("state_len", C.c_int64),
                ("kind", C.c_int32), ("coin", C.c_int32), ("dtype", C.c_int32), ("structure", C.c_int32),
                ("dims", C.c_int32 * 2), ("max_degree", C.c_int32), ("taylor_order", C.c_int32),
                ("dt", C.c_double), ("h_norm_bound", C.c_double), ("trunc_bound", C.c_double),
                ("graph_bytes", C.c_size_t), ("state_bytes", C.c_size_t), ("work_bytes", C.c_size_t),
                ("columns", C.c_int32), ("block_depth", C.c_int32)]


class QwError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2406_08186_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.qw_plan_create.argtypes = [C.POINTER(QwCsr), C.POINTER(QwWalkDesc), C.POINTER(vp)]
        L.qw_plan_destroy.argtypes = [vp]
        L.qw_plan_get_info.argtypes = [vp, C.POINTER(QwPlanInfo)]
        L.qw_plan_upload.argtypes = [vp, vp, C.c_size_t, vp]
        L.qw_evolve.argtypes = [vp, vp, vp, C.c_size_t, C.c_int64, vp, vp, vp, vp]
        L.qw_probabilities.argtypes = [vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.qw_copy_to_host.argtypes = [vp, vp, C.c_size_t, vp]
        L.qw_small_many_desc_bytes.argtypes = [C.c_int32]
        L.qw_small_many_desc_bytes.restype = C.c_size_t
        L.qw_small_many.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64), C.c_int32, vp,
                                    C.c_size_t, vp]
        L.qw_taylor_order.argtypes = [C.c_double, C.c_int64, C.c_double, C.POINTER(C.c_int32)]
        L.qw_taylor_plan.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int32),
                                     dp, C.POINTER(C.c_int64)]
        L.qw_taylor_tail_bound.argtypes = [C.c_double, C.c_int32]
        L.qw_taylor_tail_bound.restype = C.c_double
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        L.qw_batch_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(vp)]
        L.qw_batch_destroy.argtypes = [vp]
        L.qw_batch_device_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.qw_batch_bind.argtypes = [vp, vp, C.c_size_t, vp]
        L.qw_batch_set_slot.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_size_t, C.c_int64, vp]
        L.qw_batch_clear_slot.argtypes = [vp, C.c_int32]
        L.qw_batch_commit.argtypes = [vp, vp]
        L.qw_batch_run.argtypes = [vp, C.c_int64, vp]
        L.qw_batch_remaining.argtypes = [vp, C.c_int32, i64p]
        L.qw_batch_launches.argtypes = [vp, i64p]
        L.qw_batch_readout.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
        L.qw_batch_set_schedule.argtypes = [vp, C.c_int32, C.c_int32]
        L.qw_batch_autotune.argtypes = [vp, C.c_int32, vp, i32p, i32p, dp]
        L.qw_batch_set_replay.argtypes = [vp, C.c_int32]
        L.qw_batch_launch_plan.argtypes = [vp, C.c_int64, i64p, i64p]
        L.qw_batch_set_stage_kernel.argtypes = [vp, C.c_int32]
        L.qw_evolve_static.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp]
        L.qw_plan_stream_sizes.argtypes = [vp, C.c_size_t, C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                           i64p, i64p]
        L.qw_plan_upload_streamed.argtypes = [vp, C.c_size_t, C.c_int, vp, C.c_size_t, vp, C.c_size_t, vp]
        L.qw_batch_get_schedule.argtypes = [vp, i32p, i32p, i32p]
        L.qw_last_error.restype = C.c_char_p
        L.qw_version.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("qw_taylor_tail_bound", "qw_last_error", "qw_version", "qw_small_many_desc_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(code: int, fn: str) -> None:
    if code != QW_OK:
        raise QwError(code, fn, lib().qw_last_error().decode())


# ---- same-named thin wrappers ------------------------------------------------

def qw_plan_create(csr: QwCsr, desc: QwWalkDesc) -> C.c_void_p:
    out = C.c_void_p()
    check(lib().qw_plan_create(C.byref(csr), C.byref(desc), C.byref(out)), "qw_plan_create")
    return out


def qw_plan_destroy(plan) -> None:
    check(lib().qw_plan_destroy(plan), "qw_plan_destroy")


def qw_plan_get_info(plan) -> QwPlanInfo:
    info = QwPlanInfo()
    check(lib().qw_plan_get_info(plan, C.byref(info)), "qw_plan_get_info")
    return info


def qw_plan_upload(plan, d_graph: int, nbytes: int, stream: int) -> None:
    check(lib().qw_plan_upload(plan, d_graph, nbytes, stream), "qw_plan_upload")


def qw_evolve(plan, d_psi: int, d_work: int, work_bytes: int, steps: int, d_p, d_norm, d_pmarked,
              stream: int) -> None:
    check(lib().qw_evolve(plan, d_psi, d_work, work_bytes, steps, d_p, d_norm, d_pmarked, stream),
          "qw_evolve")


def qw_probabilities(plan, d_psi: int, d_p, d_norm, d_pmarked, d_work: int, work_bytes: int,
                     stream: int) -> None:
    check(lib().qw_probabilities(plan, d_psi, d_p, d_norm, d_pmarked, d_work, work_bytes, stream),
          "qw_probabilities")


def qw_copy_to_host(h_dst: int, d_src: int, nbytes: int, stream: int) -> None:
    check(lib().qw_copy_to_host(h_dst, d_src, nbytes, stream), "qw_copy_to_host")


def qw_small_many_desc_bytes(count: int) -> int:
    return int(lib().qw_small_many_desc_bytes(count))


def qw_small_many(plans, d_psi, steps, d_desc: int, desc_bytes: int, stream: int) -> None:
    n = len(plans)
    if len(d_psi) != n or len(steps) != n:
        raise ValueError("plans, states and step counts must have the same length")
    P = (C.c_void_p * max(n, 1))(*[p.value if isinstance(p, C.c_void_p) else p for p in plans])
    S = (C.c_void_p * max(n, 1))(*d_psi)
    T = (C.c_int64 * max(n, 1))(*[int(x) for x in steps])
    check(lib().qw_small_many(P, S, T, n, d_desc, desc_bytes, stream), "qw_small_many")


def qw_taylor_order(rho: float, steps: int, tol: float) -> int:
    k = C.c_int32()
    check(lib().qw_taylor_order(rho, steps, tol, C.byref(k)), "qw_taylor_order")
    return k.value


def qw_taylor_plan(h_bound: float, t_total: float, rho_max: float, tol: float):
    k, dt, n = C.c_int32(), C.c_double(), C.c_int64()
    check(lib().qw_taylor_plan(h_bound, t_total, rho_max, tol, C.byref(k), C.byref(dt), C.byref(n)),
          "qw_taylor_plan")
    return k.value, dt.value, n.value


def qw_taylor_tail_bound(rho: float, K: int) -> float:
    return float(lib().qw_taylor_tail_bound(rho, K))


def qw_version() -> str:
    return lib().qw_version().decode()


# ---- batches --------------------------------------------------------------------

def qw_batch_create(capacity: int, max_tiles: int, dtype: int) -> C.c_void_p:
    out = C.c_void_p()
    check(lib().qw_batch_create(capacity, max_tiles, dtype, C.byref(out)), "qw_batch_create")
    return out


def qw_batch_destroy(batch) -> None:
    check(lib().qw_batch_destroy(batch), "qw_batch_destroy")


def qw_batch_device_bytes(batch) -> int:
    n = C.c_size_t()
    check(lib().qw_batch_device_bytes(batch, C.byref(n)), "qw_batch_device_bytes")
    return n.value


def qw_batch_bind(batch, d_buf: int, nbytes: int, stream: int) -> None:
    check(lib().qw_batch_bind(batch, d_buf, nbytes, stream), "qw_batch_bind")


def qw_batch_set_slot(batch, slot: int, plan, d_psi: int, d_work: int, work_bytes: int, steps: int,
                      d_hist) -> None:
    check(lib().qw_batch_set_slot(batch, slot, plan, d_psi, d_work, work_bytes, steps, d_hist),
          "qw_batch_set_slot")


def qw_batch_clear_slot(batch, slot: int) -> None:
    check(lib().qw_batch_clear_slot(batch, slot), "qw_batch_clear_slot")


def qw_batch_commit(batch, stream: int) -> None:
    check(lib().qw_batch_commit(batch, stream), "qw_batch_commit")


def qw_batch_run(batch, launches: int, stream: int) -> None:
    check(lib().qw_batch_run(batch, launches, stream), "qw_batch_run")


def qw_batch_remaining(batch, slot: int) -> int:
    r = C.c_int64()
    check(lib().qw_batch_remaining(batch, slot, C.byref(r)), "qw_batch_remaining")
    return r.value


def qw_batch_launches(batch) -> int:
    r = C.c_int64()
    check(lib().qw_batch_launches(batch, C.byref(r)), "qw_batch_launches")
    return r.value


def qw_batch_readout(batch, slot: int, d_p, d_norm, d_pmarked, stream: int) -> None:
    check(lib().qw_batch_readout(batch, slot, d_p, d_norm, d_pmarked, stream), "qw_batch_readout")


def qw_batch_set_schedule(batch, rows_per_tile: int, xcd_aware: int) -> None:
    check(lib().qw_batch_set_schedule(batch, rows_per_tile, xcd_aware), "qw_batch_set_schedule")


def qw_batch_set_replay(batch, use_graph: int) -> None:
    check(lib().qw_batch_set_replay(batch, use_graph), "qw_batch_set_replay")


def qw_batch_launch_plan(batch, launches: int) -> tuple[int, int]:
    g, d = C.c_int64(), C.c_int64()
    check(lib().qw_batch_launch_plan(batch, launches, C.byref(g), C.byref(d)), "qw_batch_launch_plan")
    return g.value, d.value


QW_STATIC_SCRATCH_BYTES = 64 * 1024 * 1024


def qw_evolve_static(plan, d_psi: int, steps: int, d_p, d_norm, d_pmarked, stream: int) -> None:
    check(lib().qw_evolve_static(plan, d_psi, steps, d_p, d_norm, d_pmarked, stream), "qw_evolve_static")


def qw_plan_stream_sizes(plan, device_budget: int, mode: int = 0) -> tuple[int, int, int, int]:
    h, d, t, a = C.c_size_t(), C.c_size_t(), C.c_int64(), C.c_int64()
    check(lib().qw_plan_stream_sizes(plan, device_budget, mode, C.byref(h), C.byref(d), C.byref(t), C.byref(a)),
          "qw_plan_stream_sizes")
    return h.value, d.value, t.value, a.value


def qw_plan_upload_streamed(plan, device_budget: int, mode: int, h_pinned: int, host_bytes: int, d_buf: int,
                            device_bytes: int, stream: int) -> None:
    check(lib().qw_plan_upload_streamed(plan, device_budget, mode, h_pinned, host_bytes, d_buf, device_bytes,
                                        stream),
          "qw_plan_upload_streamed")


def qw_batch_set_stage_kernel(batch, kernel: int) -> None:
    check(lib().qw_batch_set_stage_kernel(batch, kernel), "qw_batch_set_stage_kernel")


def qw_batch_get_schedule(batch) -> tuple[int, int, int]:
    r, x, k = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().qw_batch_get_schedule(batch, C.byref(r), C.byref(x), C.byref(k)), "qw_batch_get_schedule")
    return r.value, x.value, k.value


def qw_batch_autotune(batch, reps: int, stream: int):
    r, x, ms = C.c_int32(), C.c_int32(), C.c_double()
    check(lib().qw_batch_autotune(batch, reps, stream, C.byref(r), C.byref(x), C.byref(ms)),
          "qw_batch_autotune")
    return r.value, x.value, ms.value
