"""Python surface of the engine: plans over torch device memory, and the
user-level walk classes modelled on Hiperwalk's frontend (Sec. 3.1, 3.2).

Torch owns every device buffer and stream; the library only enqueues
kernels on the stream it is given.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Iterable, Sequence

import numpy as np
import torch

from . import _lib as L
from .inputs import Graph, arc_index

_DT = {"c64": L.QW_C64, "c128": L.QW_C128}
_TORCH_DT = {"c64": torch.complex64, "c128": torch.complex128}
_LAYOUT = {"auto": L.QW_LAYOUT_AUTO, "csr": L.QW_LAYOUT_CSR, "structured": L.QW_LAYOUT_STRUCTURED,
           "dense": L.QW_LAYOUT_DENSE}


def _stream_ptr(stream, device) -> int:
    """Handle of the stream to launch on (default: torch's current stream).  A
    different stream first waits for the current one, so buffers that torch
    allocated or filled there are ready before the launch reads or writes them."""
    cur = torch.cuda.current_stream(device)
    if stream is None or stream.cuda_stream == cur.cuda_stream:
        return int(cur.cuda_stream)
    stream.wait_stream(cur)
    return int(stream.cuda_stream)


class Plan:
    """A validated walk on one graph with its device tables uploaded.

    kind: "coined", "ctqw" or "staggered" (with `tessellations`, a sequence of
    objects with poly_ptr, poly_vert, amp (None = uniform) and theta (None =
    reflection form)); coin: "grover", "hadamard", "fourier", "szegedy"
    (with `transition`, P per arc in CSR order) or a d x d complex matrix;
    shift: "flipflop" or "persistent"; dtype: "c64" or "c128";
    layout: "auto", "csr", "structured" or "dense".  CTQW takes gamma, dt and
    either taylor_order or (trunc_tol, horizon_steps); the dense layout takes
    `columns` walks sharing H (state n x columns, vertex-major).
    """

    def __init__(self, graph: Graph, kind: str = "coined", *, coin="grover", shift: str = "flipflop",
                 dtype: str = "c128", layout: str = "auto", gamma: float = 0.0, dt: float = 0.0,
                 taylor_order: int = 0, trunc_tol: float = 0.0, horizon_steps: int = 0,
                 marked: Sequence[int] = (), columns: int = 0, device=None, stream=None,
                 upload: bool = True, transition=None, tessellations=None):
        self.graph = graph
        self.kind = kind
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self._rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int64)
        self._col = np.ascontiguousarray(graph.col, dtype=np.int32)
        if self._col.size == 0:
            self._col = np.zeros(1, dtype=np.int32)
        self._marked = np.ascontiguousarray(np.asarray(list(marked), dtype=np.int32))
        self._trans = None
        if isinstance(coin, str):
            coin_id = {"grover": L.QW_GROVER, "hadamard": L.QW_HADAMARD, "fourier": L.QW_FOURIER,
                       "szegedy": L.QW_SZEGEDY}[coin]
            self._coin = None
            if coin == "szegedy":
                if transition is None:
                    raise ValueError("the Szegedy coin needs transition (P per arc, CSR order)")
                self._trans = np.ascontiguousarray(np.asarray(transition, dtype=np.float64))
        else:
            coin_id = L.QW_MATRIX
            self._coin = np.ascontiguousarray(np.asarray(coin, dtype=np.complex128))
            if self._coin.ndim != 2 or self._coin.shape[0] != self._coin.shape[1]:
                raise ValueError("a coin matrix must be square")
        n_tess, tess_arr = 0, None
        if kind == "staggered":
            if not tessellations:
                raise ValueError("a staggered walk needs tessellations")
            self._tess_keep = []
            tess_arr = (L.QwTessellation * len(tessellations))()
            for i, t in enumerate(tessellations):
                pp = np.ascontiguousarray(t.poly_ptr, dtype=np.int64)
                vv = np.ascontiguousarray(t.poly_vert, dtype=np.int32)
                aa = None if t.amp is None else np.ascontiguousarray(t.amp, dtype=np.float64)
                self._tess_keep += [pp, vv, aa]
                tess_arr[i] = L.QwTessellation(
                    n_polygons=int(pp.size - 1), poly_ptr=pp.ctypes.data_as(C.POINTER(C.c_int64)),
                    poly_vert=vv.ctypes.data_as(C.POINTER(C.c_int32)),
                    amp=None if aa is None else aa.ctypes.data_as(C.POINTER(C.c_double)),
                    form=L.QW_REFLECTION if t.theta is None else L.QW_HAMILTONIAN,
                    theta=0.0 if t.theta is None else float(t.theta))
            n_tess = len(tessellations)
        elif kind not in ("coined", "ctqw"):
            raise ValueError(f"unknown walk kind {kind!r}")
        csr = L.QwCsr(graph.n, self._rp.ctypes.data_as(C.POINTER(C.c_int64)),
                      self._col.ctypes.data_as(C.POINTER(C.c_int32)))
        desc = L.QwWalkDesc(
            kind={"coined": L.QW_COINED, "ctqw": L.QW_CTQW, "staggered": L.QW_STAGGERED}[kind],
            coin=coin_id,
            dtype=_DT[dtype], layout=_LAYOUT[layout], gamma=float(gamma), dt=float(dt),
            taylor_order=int(taylor_order), trunc_tol=float(trunc_tol),
            horizon_steps=int(horizon_steps),
            marked=self._marked.ctypes.data_as(C.POINTER(C.c_int32)) if self._marked.size else None,
            n_marked=int(self._marked.size), columns=int(columns),
            shift={"flipflop": L.QW_FLIPFLOP, "persistent": L.QW_PERSISTENT}[shift],
            coin_dim=0 if self._coin is None else int(self._coin.shape[0]),
            coin_matrix=None if self._coin is None else self._coin.view(np.float64).ctypes.data_as(
                C.POINTER(C.c_double)),
            transition=None if self._trans is None else self._trans.ctypes.data_as(C.POINTER(C.c_double)),
            n_tessellations=n_tess, tessellations=tess_arr)
        self._plan = L.qw_plan_create(csr, desc)
        self.info = L.qw_plan_get_info(self._plan)
        self.structure = L.STRUCTURES[self.info.structure]
        self.d_graph = None
        if upload:
            self.upload(stream)

    @property
    def device_bytes(self) -> int:
        """Device memory this plan needs once uploaded: tables, workspace, one state."""
        return int(self.info.graph_bytes + self.info.work_bytes + self.info.state_bytes)

    def upload(self, stream=None) -> None:
        """Allocate the device tables and workspace (torch) and upload (second phase)."""
        self.d_graph = torch.empty(max(self.info.graph_bytes, 256), dtype=torch.uint8, device=self.device)
        self.work = torch.empty(max(self.info.work_bytes, 256), dtype=torch.uint8, device=self.device)
        self._p = torch.empty(max(self.p_len, 1), dtype=torch.float64, device=self.device)
        self._scal = torch.zeros(2, dtype=torch.float64, device=self.device)
        L.qw_plan_upload(self._plan, self.d_graph.data_ptr(), self.d_graph.numel(),
                         _stream_ptr(stream, self.device))

    def upload_streamed(self, device_budget: int, mode: str = "direct", stream=None) -> dict:
        """Out-of-core binding (CTQW on the CSR layout): the neighbour table goes to a
        pinned host buffer; the walk uses at most `device_budget` bytes of device
        memory.  mode "direct": the device keeps what fits of the table and the
        stage kernel reads the rest from host memory; "ring": the table streams
        through a ring of device slots at every Horner stage."""
        m = {"direct": L.QW_STREAM_DIRECT, "ring": L.QW_STREAM_RING}[mode]
        host_bytes, dev_bytes, tiles, dev_arcs = L.qw_plan_stream_sizes(self._plan, int(device_budget), m)
        self.h_graph = torch.empty(max(host_bytes, 256), dtype=torch.uint8, pin_memory=True)
        self.d_graph = torch.empty(max(dev_bytes, 256), dtype=torch.uint8, device=self.device)
        self.work = torch.empty(max(self.info.work_bytes, 256), dtype=torch.uint8, device=self.device)
        self._p = torch.empty(max(self.p_len, 1), dtype=torch.float64, device=self.device)
        self._scal = torch.zeros(2, dtype=torch.float64, device=self.device)
        L.qw_plan_upload_streamed(self._plan, int(device_budget), m, self.h_graph.data_ptr(), self.h_graph.numel(),
                                  self.d_graph.data_ptr(), self.d_graph.numel(), _stream_ptr(stream, self.device))
        return {"host_bytes": host_bytes, "device_bytes": dev_bytes, "tiles": tiles, "device_arcs": dev_arcs,
                "mode": mode}

    def release_device(self) -> None:
        """Drop the device buffers (the plan must not be used on the device afterwards)."""
        self.d_graph = self.work = self._p = self._scal = None

    # -- lifetime
    def close(self) -> None:
        if getattr(self, "_plan", None):
            L.qw_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- states
    @property
    def state_len(self) -> int:
        return int(self.info.state_len)

    @property
    def p_len(self) -> int:
        """Length of the probability readout: n, or n * columns for the dense layout."""
        return int(self.graph.n * max(1, self.info.columns))

    def state(self, psi0) -> torch.Tensor:
        """Device copy of psi0 in this plan's precision."""
        t = torch.as_tensor(np.asarray(psi0) if not torch.is_tensor(psi0) else psi0)
        if t.numel() != self.state_len:
            raise ValueError(f"state has {t.numel()} elements, plan needs {self.state_len}")
        return t.to(device=self.device, dtype=_TORCH_DT[self.dtype]).contiguous()

    def _check(self, psi: torch.Tensor) -> None:
        if psi.device != self.device or psi.dtype != _TORCH_DT[self.dtype] or not psi.is_contiguous() \
                or psi.numel() != self.state_len:
            raise ValueError("state tensor does not match the plan (device/dtype/length/contiguity)")

    # -- hot path
    def evolve(self, psi: torch.Tensor, steps: int, readout: bool = False, stream=None):
        """psi <- U^steps psi in place; with readout, also (p, norm, p_marked) on device."""
        self._check(psi)
        sp = _stream_ptr(stream, self.device)
        if readout:
            p, scal = self._p, self._scal
            L.qw_evolve(self._plan, psi.data_ptr(), self.work.data_ptr(), self.work.numel(), int(steps),
                        p.data_ptr(), scal.data_ptr(), scal.data_ptr() + 8, sp)
            return p[:self.p_len], scal[0], scal[1]
        L.qw_evolve(self._plan, psi.data_ptr(), self.work.data_ptr(), self.work.numel(), int(steps),
                    None, None, None, sp)
        return None

    def probabilities(self, psi: torch.Tensor, stream=None):
        """(p, norm, p_marked) of a state, FP64, on device."""
        self._check(psi)
        p = torch.empty(max(self.p_len, 1), dtype=torch.float64, device=self.device)
        scal = torch.zeros(2, dtype=torch.float64, device=self.device)
        L.qw_probabilities(self._plan, psi.data_ptr(), p.data_ptr(), scal.data_ptr(),
                           scal.data_ptr() + 8, self.work.data_ptr(), self.work.numel(),
                           _stream_ptr(stream, self.device))
        return p[:self.p_len], scal[0], scal[1]


def evolve_many(plans: Sequence["Plan"], states: Sequence[torch.Tensor], steps: Sequence[int],
                stream=None) -> torch.Tensor:
    """Advance many small walks (plans on the one-workgroup path, one dtype) by
    their step counts in one launch (qw_small_many).  Returns the device buffer
    holding the walk descriptors; keep it until the launch has run."""
    if not (len(plans) == len(states) == len(steps)):
        raise ValueError("plans, states and step counts must have the same length")
    for pl, psi in zip(plans, states):
        pl._check(psi)
    dev = plans[0].device if plans else torch.device("cuda", 0)
    nbytes = L.qw_small_many_desc_bytes(len(plans))
    desc = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    L.qw_small_many([pl._plan for pl in plans], [psi.data_ptr() for psi in states], list(steps),
                    desc.data_ptr(), desc.numel(), _stream_ptr(stream, dev))
    return desc


class Batch:
    """Many walks advanced together (qw_batch_*): slots hold (plan, state, steps).

    Plans must use layout "csr".  Each slot keeps references to its plan, state
    and history tensors until it is cleared.
    """

    def __init__(self, capacity: int, max_tiles: int, dtype: str = "c64", device=None, stream=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.dtype = dtype
        self.capacity = capacity
        self._b = L.qw_batch_create(capacity, max_tiles, _DT[dtype])
        nbytes = L.qw_batch_device_bytes(self._b)
        self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        L.qw_batch_bind(self._b, self.buf.data_ptr(), self.buf.numel(), _stream_ptr(stream, self.device))
        self._held = {}

    def close(self) -> None:
        if getattr(self, "_b", None):
            L.qw_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_slot(self, slot: int, plan: Plan, psi: torch.Tensor, steps: int,
                 hist: torch.Tensor | None = None) -> None:
        plan._check(psi)
        if hist is not None and (hist.dtype != torch.float64 or hist.numel() < steps
                                 or hist.device != self.device):
            raise ValueError("hist must be a float64 device tensor of at least `steps` elements")
        L.qw_batch_set_slot(self._b, slot, plan._plan, psi.data_ptr(), plan.work.data_ptr(),
                            plan.work.numel(), int(steps), hist.data_ptr() if hist is not None else None)
        self._held[slot] = (plan, psi, hist)

    def clear_slot(self, slot: int) -> None:
        L.qw_batch_clear_slot(self._b, slot)
        self._held.pop(slot, None)

    def commit(self, stream=None) -> None:
        L.qw_batch_commit(self._b, _stream_ptr(stream, self.device))

    def run(self, launches: int, stream=None) -> None:
        L.qw_batch_run(self._b, int(launches), _stream_ptr(stream, self.device))

    def set_replay(self, use_graph: bool) -> None:
        """Graph replay (default) or direct launches for qw_batch_run (same kernels and results)."""
        L.qw_batch_set_replay(self._b, int(bool(use_graph)))

    def remaining(self, slot: int) -> int:
        return L.qw_batch_remaining(self._b, slot)

    @property
    def launches(self) -> int:
        return L.qw_batch_launches(self._b)

    def active_slots(self) -> list[int]:
        return sorted(self._held)

    def run_to_completion(self, stream=None) -> int:
        n = max((self.remaining(s) for s in self._held), default=0)
        self.run(n, stream)
        return n

    def readout(self, slot: int, stream=None):
        plan = self._held[slot][0]
        p = torch.empty(max(plan.graph.n, 1), dtype=torch.float64, device=self.device)
        scal = torch.zeros(2, dtype=torch.float64, device=self.device)
        L.qw_batch_readout(self._b, slot, p.data_ptr(), scal.data_ptr(), scal.data_ptr() + 8,
                           _stream_ptr(stream, self.device))
        return p[:plan.graph.n], scal[0], scal[1]

    def set_schedule(self, rows_per_tile: int, xcd_aware: bool = True) -> None:
        L.qw_batch_set_schedule(self._b, rows_per_tile, int(xcd_aware))

    def set_stage_kernel(self, kernel: str) -> None:
        """"lds" (default) or "gather" for CTQW walks on regular graphs of degree <= 8
        (takes effect at the next commit)."""
        L.qw_batch_set_stage_kernel(self._b, {"gather": L.QW_BATCH_GATHER, "lds": L.QW_BATCH_LDS}[kernel])

    def schedule(self) -> dict:
        r, x, k = L.qw_batch_get_schedule(self._b)
        return {"rows_per_tile": r, "xcd_aware": bool(x), "stage_kernel": "lds" if k == L.QW_BATCH_LDS else "gather"}

    def autotune(self, reps: int = 3, stream=None):
        return L.qw_batch_autotune(self._b, reps, _stream_ptr(stream, self.device))


def _steps_of(rng) -> list[int]:
    if isinstance(rng, int):
        return list(range(rng))
    if isinstance(rng, range):
        return list(rng)
    return list(range(*rng))


def stream_snapshots(plan: Plan, psi: torch.Tensor, steps: Sequence[int], kind: str = "state",
                     ring: int = 3, host: Sequence[torch.Tensor] | None = None,
                     via: str = "link") -> list[np.ndarray]:
    """Evolve psi in place through the step indices `steps` (increasing, from the
    state's current step 0) and return, for each, the state (kind "state") or
    its FP64 vertex probabilities (kind "probability") in host memory.

    via "link" (the default): on torch's current stream, after the evolve that
    reaches each step, qw_copy_to_host writes the state (or the
    qw_probabilities readout) straight into the pinned host buffer with a
    kernel, ordered with the walk like any other launch.  via "memcpy": each
    snapshot is copied into one of `ring` device slots and from there to the
    host buffer by the runtime's asynchronous copy on a second stream while
    the walk moves on; a slot is reused only after its copy has finished.  Either way the
    snapshots equal those of evolve calls stopped at each step (the same
    kernels run).  `host` may supply the pinned, contiguous destination
    tensors (one per step) for reuse."""
    if kind not in ("state", "probability"):
        raise ValueError("kind is 'state' or 'probability'")
    if via not in ("link", "memcpy"):
        raise ValueError("via is 'link' or 'memcpy'")
    steps = list(steps)
    if any(b <= a for a, b in zip(steps, steps[1:])) or (steps and steps[0] < 0):
        raise ValueError("steps must be increasing and non-negative")
    plan._check(psi)
    dev = plan.device
    cs = torch.cuda.current_stream(dev)
    shape, dt = (psi.shape, psi.dtype) if kind == "state" else ((plan.p_len,), torch.float64)
    if host is None:
        host = [torch.empty(shape, dtype=dt, pin_memory=True) for _ in steps]
    elif len(host) != len(steps) or any(h.shape != shape or h.dtype != dt or not h.is_pinned()
                                        or not h.is_contiguous() for h in host):
        raise ValueError("host buffers must be pinned and contiguous, one per step, of the snapshot's "
                         "shape and dtype")
    if via == "link":
        if kind == "probability":
            pbuf = torch.empty(max(plan.p_len, 1), dtype=torch.float64, device=dev)
            scal = torch.empty(2, dtype=torch.float64, device=dev)
        at = 0
        for j, k in enumerate(steps):
            plan.evolve(psi, k - at, stream=cs)
            at = k
            if kind == "state":
                src = psi
            else:
                L.qw_probabilities(plan._plan, psi.data_ptr(), pbuf.data_ptr(), scal.data_ptr(), None,
                                   plan.work.data_ptr(), plan.work.numel(), int(cs.cuda_stream))
                src = pbuf
            L.qw_copy_to_host(host[j].data_ptr(), src.data_ptr(), host[j].numel() * host[j].element_size(),
                              int(cs.cuda_stream))
        cs.synchronize()
        return [h.numpy() for h in host]
    xs = torch.cuda.Stream(dev)
    if kind == "state":
        slots = [torch.empty_like(psi) for _ in range(ring)]
    else:
        slots = [torch.empty(max(plan.p_len, 1), dtype=torch.float64, device=dev) for _ in range(ring)]
        scal = torch.empty(2, dtype=torch.float64, device=dev)
    free = [None] * ring
    at = 0
    for j, k in enumerate(steps):
        plan.evolve(psi, k - at, stream=cs)
        at = k
        slot = j % ring
        if free[slot] is not None:
            cs.wait_event(free[slot])
        if kind == "state":
            slots[slot].copy_(psi)
        else:
            L.qw_probabilities(plan._plan, psi.data_ptr(), slots[slot].data_ptr(), scal.data_ptr(), None,
                               plan.work.data_ptr(), plan.work.numel(), int(cs.cuda_stream))
        ready = torch.cuda.Event()
        ready.record(cs)
        xs.wait_event(ready)
        with torch.cuda.stream(xs):
            host[j].copy_(slots[slot][:host[j].numel()], non_blocking=True)
        free[slot] = torch.cuda.Event()
        free[slot].record(xs)
    xs.synchronize()
    return [h.numpy() for h in host]


class _Walk:
    plan: Plan

    def simulate(self, range=1, state=None) -> list[torch.Tensor]:
        """States at the step indices of Python's range(...) (snapshots include step 0
        when the range starts at 0).  Returns device tensors."""
        idx = _steps_of(range)
        if any(b <= a for a, b in zip(idx, idx[1:])) or (idx and idx[0] < 0):
            raise ValueError("range must be increasing and non-negative")
        psi = self.plan.state(state)
        out, at = [], 0
        for k in idx:
            self.plan.evolve(psi, k - at)
            at = k
            out.append(psi.clone())
        return out

    def probability_distribution(self, states: Iterable[torch.Tensor]) -> list[torch.Tensor]:
        return [self.plan.probabilities(s)[0].clone() for s in states]

    def simulate_host(self, range=1, state=None, kind: str = "state") -> list[np.ndarray]:
        """simulate() streamed to host memory: states (or, with kind
        "probability", FP64 distributions) at the step indices of range(...),
        written into pinned host memory by a copy kernel on the walk's stream
        as each step is reached."""
        psi = self.plan.state(state)
        return stream_snapshots(self.plan, psi, _steps_of(range), kind)


class Coined(_Walk):
    """Coined walk U = S C (Sec. 3.2): flip-flop shift on any graph, or the
    persistent shift on cycles and periodic grids; Grover, Hadamard, Fourier, a
    caller's coin matrix, or Szegedy's reflection for a transition matrix P
    (Szegedy's walk, Sec. 5)."""

    def __init__(self, graph: Graph, shift: str = "flipflop", coin="grover",
                 marked: Sequence[int] = (), dtype: str = "c128", layout: str = "auto", device=None,
                 transition=None):
        self.graph = graph
        self.plan = Plan(graph, "coined", coin=coin, shift=shift, dtype=dtype, layout=layout,
                         marked=marked, device=device, transition=transition)

    def ket(self, v: int, w: int) -> np.ndarray:
        psi = np.zeros(self.graph.n_arcs, dtype=np.complex128)
        psi[arc_index(self.graph, v, w)] = 1.0
        return psi


class ContinuousTime(_Walk):
    """Continuous-time walk, H = -gamma A - sum_M |v><v| (Sec. 3.1); `time` is the
    step length of simulate()."""

    def __init__(self, graph: Graph, gamma: float, time: float, marked: Sequence[int] = (),
                 dtype: str = "c128", taylor_order: int = 0, trunc_tol: float = 1e-13,
                 horizon_steps: int = 10**4, layout: str = "auto", device=None):
        self.graph = graph
        self.gamma = gamma
        self.marked = list(marked)
        self.plan = Plan(graph, "ctqw", dtype=dtype, layout=layout, gamma=gamma, dt=time,
                         taylor_order=taylor_order, trunc_tol=trunc_tol,
                         horizon_steps=horizon_steps, marked=marked, device=device)

    def ket(self, v: int) -> np.ndarray:
        psi = np.zeros(self.graph.n, dtype=np.complex128)
        psi[v] = 1.0
        return psi

    def get_hamiltonian(self):
        """H as (row_ptr, col, value of the off-diagonal -gamma, diagonal marked list)."""
        return self.graph.row_ptr, self.graph.col, -self.gamma, list(self.marked)


class Staggered(_Walk):
    """Staggered walk (named as future work in Sec. 5): one step is the
    marked vertices' phase flip followed by U_k = 2 P_k - I (or
    exp(i theta_k (2 P_k - I))) for each tessellation in order, on the
    vertex basis.  Every polygon must be a clique of `graph`."""

    def __init__(self, graph: Graph, tessellations, marked: Sequence[int] = (), dtype: str = "c128",
                 layout: str = "auto", device=None):
        self.graph = graph
        self.tessellations = list(tessellations)
        self.plan = Plan(graph, "staggered", dtype=dtype, layout=layout, marked=marked, device=device,
                         tessellations=self.tessellations)

    def ket(self, v: int) -> np.ndarray:
        psi = np.zeros(self.graph.n, dtype=np.complex128)
        psi[v] = 1.0
        return psi


def uniform_state(n: int) -> np.ndarray:
    return np.full(n, 1.0 / math.sqrt(n), dtype=np.complex128)
