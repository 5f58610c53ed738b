"""Python binding of libvmo (include/vmo.h): geometric matrix ordering on MI355X.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libvmo.so``.  PyTorch supplies device memory (tensors) and the current
HIP stream.  If the library is not built this module raises at first use;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
from collections.abc import Mapping
import functools
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvmo.so")

VMO_OK, VMO_E_INVALID, VMO_E_NOMEM, VMO_E_DEVICE, VMO_E_UNSUPPORTED, VMO_E_BUSY = 0, -1, -2, -3, -4, -5
ROW_NET, COLUMN_NET, SYMMETRIC, BIPARTITE = 0, 1, 2, 3
NET, GRAPH = 0, 1
SBD, BBD = 0, 1


class VmoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"vmo status {status}: {msg}")
        self.status = status


class Hypergraph(C.Structure):
    _fields_ = [("k", C.c_int32), ("l", C.c_int32), ("net_ptr", C.c_void_p), ("pins", C.c_void_p),
                ("w", C.c_void_p), ("c", C.c_void_p)]


class LayoutParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("coarsest_iters", C.c_int32), ("level_iters", C.c_int32),
                ("min_coarse", C.c_int32), ("max_levels", C.c_int32), ("leaf_cap", C.c_int32),
                ("match_max_net", C.c_int32), ("theta", C.c_float), ("step0_frac", C.c_float),
                ("decay", C.c_float), ("jitter", C.c_float), ("stall", C.c_float), ("pack_gap", C.c_float)]


class OrderOut(C.Structure):
    _fields_ = [("vperm", C.c_void_p), ("nperm", C.c_void_p), ("part", C.c_void_p), ("node_heap", C.c_void_p),
                ("node_vptr", C.c_void_p), ("node_nptr", C.c_void_p), ("split_cut", C.c_void_p),
                ("n_nodes", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("h", Hypergraph), ("mode", C.c_int32), ("order", C.c_int32), ("x", C.c_void_p), ("P", C.c_int32),
                ("seed", C.c_uint64), ("job_index", C.c_uint64), ("out", OrderOut)]


@functools.lru_cache(maxsize=1)
def _job_dtype():
    """numpy record type with the memory layout of vmo_job (from the ctypes
    definition), for filling many jobs at once."""
    import numpy as np
    names, fmts, offsets = [], [], []
    for f, t in Hypergraph._fields_:
        names.append(f)
        fmts.append(np.int32 if t is C.c_int32 else np.uint64)
        offsets.append(Job.h.offset + getattr(Hypergraph, f).offset)
    for f in ("mode", "order", "x", "P", "seed", "job_index"):
        names.append(f)
        fmts.append(np.int32 if f in ("mode", "order", "P") else np.uint64)
        offsets.append(getattr(Job, f).offset)
    for f, _ in OrderOut._fields_:
        names.append("o_" + f)
        fmts.append(np.uint64)
        offsets.append(Job.out.offset + getattr(OrderOut, f).offset)
    return np.dtype({"names": names, "formats": fmts, "offsets": offsets, "itemsize": C.sizeof(Job)})


class ProfileEntry(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("launches", C.c_int64), ("work", C.c_double)]


class ServeParams(C.Structure):
    _fields_ = [("device", C.c_int), ("budget_bytes", C.c_size_t), ("max_jobs", C.c_int32), ("t_max", C.c_int32),
                ("layout_threads", C.c_int32)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("ticks", C.c_int64), ("resident", C.c_int64),
                ("pending", C.c_int64), ("busy_ms", C.c_double), ("capacity_vertices", C.c_int64),
                ("capacity_pins", C.c_int64), ("capacity_edges", C.c_int64), ("max_tick_jobs", C.c_int64),
                ("tick_jobs", C.c_int64), ("layout_budget_bytes", C.c_int64), ("layout_bytes_peak", C.c_int64)]


class CutResult(C.Structure):
    _fields_ = [("lambda_minus_one", C.c_double), ("cut_net", C.c_double), ("nets_cut", C.c_int64),
                ("max_split", C.c_double), ("max_split_node", C.c_int32), ("separators", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1105_4490_amd.build` "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.vmo_last_error.restype = C.c_char_p
        L.vmo_pool_bytes.restype = C.c_size_t
        L.vmo_serve_error.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def layout_params(seed=1, **kw) -> LayoutParams:
    p = LayoutParams()
    lib().vmo_layout_defaults(C.byref(p), C.c_uint64(seed))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@dataclass
class DeviceHypergraph:
    """A hypergraph whose arrays live on the GPU (Definition of a hypergraph, Sec. 1.1)."""
    k: int
    l: int
    net_ptr: torch.Tensor   # int64 [l+1]
    pins: torch.Tensor      # int32
    w: torch.Tensor | None = None
    c: torch.Tensor | None = None

    def cstruct(self) -> Hypergraph:
        return Hypergraph(self.k, self.l, _ptr(self.net_ptr), _ptr(self.pins) if self.pins.numel() else None,
                          _ptr(self.w), _ptr(self.c))

    def cptrs(self):
        """Device addresses (net_ptr, pins, w, c); 0 for an absent array."""
        return (self.net_ptr.data_ptr(), self.pins.data_ptr() if self.pins.numel() else 0,
                self.w.data_ptr() if self.w is not None else 0, self.c.data_ptr() if self.c is not None else 0)

    @staticmethod
    def from_host(h, device="cuda"):
        """From any object with k, l, ptr/net_ptr, pins, w, c (numpy arrays)."""
        ptr = getattr(h, "ptr", None)
        if ptr is None:
            ptr = h.net_ptr
        t = lambda a, dt: None if a is None else torch.as_tensor(a, dtype=dt).to(device).contiguous()
        pins = t(h.pins, torch.int32)
        if pins.numel() == 0:
            pins = torch.zeros(1, dtype=torch.int32, device=device)
        return DeviceHypergraph(int(h.k), int(h.l), t(ptr, torch.int64), pins, t(getattr(h, "w", None), torch.float32),
                                t(getattr(h, "c", None), torch.float32))


class _BatchOut(Mapping):
    """Outputs of one job of a batch: views into the batch's shared arrays,
    formed when read (a batch of hundreds of jobs would otherwise spend
    milliseconds forming views that are never used)."""
    __slots__ = ("_flat", "_sz", "_off", "_i", "_net", "_l")

    def __init__(self, flat, sz, off, i, net, l):
        self._flat, self._sz, self._off, self._i, self._net, self._l = flat, sz, off, i, net, l

    def __getitem__(self, f):
        if f not in self._flat:
            raise KeyError(f)
        if not self._net and f in ("nperm", "node_nptr"):
            return None
        n = self._l if f == "nperm" else self._sz[f][self._i]
        return self._flat[f].narrow(0, self._off[f][self._i], n)

    def __iter__(self):
        return iter(self._flat)

    def __len__(self):
        return len(self._flat)


class Context:
    """One vmo context on one GPU (calls on it must not overlap)."""

    def __init__(self, device: int | None = None, pool_bytes: int = 0):
        self.device = torch.cuda.current_device() if device is None else device
        h = C.c_void_p()
        self._check(lib().vmo_create(C.byref(h), C.c_int(self.device), C.c_size_t(pool_bytes)), ctx=None)
        self.h = h

    def sync(self, stream=None):
        """vmo_sync: waits for the stream's work and reports what the device-
        side checks of earlier asynchronous calls found (raises VmoError)."""
        st = _stream() if stream is None else C.c_void_p(stream.cuda_stream)
        self._check(lib().vmo_sync(self.h, st))

    def close(self):
        if getattr(self, "h", None):
            lib().vmo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ctx="self"):
        if st != VMO_OK:
            msg = lib().vmo_last_error(self.h).decode() if ctx is not None else "vmo_create failed"
            raise VmoError(st, msg)

    @staticmethod
    def layout_bytes(k: int, l: int, npins: int) -> int:
        """vmo_layout_bytes: bound of vmo_layout's workspace for these sizes."""
        lib().vmo_layout_bytes.restype = C.c_size_t
        return int(lib().vmo_layout_bytes(C.c_int32(k), C.c_int32(l), C.c_int64(npins)))

    def pool_bytes(self) -> int:
        return int(lib().vmo_pool_bytes(self.h))

    def profile(self, enable, every: int = 1, count: bool = True):
        """Live kernel timing with HIP events on the launch stream: off when
        enable is false, else every `every`-th launch of each kernel is timed;
        count=False leaves out the work the kernels count on the device (the
        walk runs uncounted)."""
        n = int(every) if count else -int(every)
        self._check(lib().vmo_profile(self.h, C.c_int(n if enable else 0)))

    def profile_reset(self):
        self._check(lib().vmo_profile_reset(self.h))

    def profile_read(self, kernel: str):
        e = ProfileEntry()
        self._check(lib().vmo_profile_read(self.h, kernel.encode(), C.byref(e)))
        return {"total_ms": e.total_ms, "launches": e.launches, "work": e.work}

    # --------------------------------------------------------------- models --
    def model(self, kind: int, m: int, n: int, rowptr: torch.Tensor, col: torch.Tensor) -> DeviceHypergraph:
        nnz = int(col.numel())
        cap_nets = {ROW_NET: m, COLUMN_NET: n, SYMMETRIC: max(nnz, 1), BIPARTITE: nnz}[kind]
        cap_pins = {ROW_NET: nnz, COLUMN_NET: nnz, SYMMETRIC: 2 * nnz, BIPARTITE: 2 * nnz}[kind]
        dev = rowptr.device
        net_ptr = torch.empty(cap_nets + 1, dtype=torch.int64, device=dev)
        pins = torch.empty(max(cap_pins, 1), dtype=torch.int32, device=dev)
        k, l, npins = C.c_int32(), C.c_int32(), C.c_int64()
        self._check(lib().vmo_model(self.h, C.c_int(kind), C.c_int32(m), C.c_int32(n), _ptr(rowptr),
                                    _ptr(col) if nnz else None, _ptr(net_ptr), _ptr(pins), C.c_int32(cap_nets),
                                    C.c_int64(cap_pins), C.byref(k), C.byref(l), C.byref(npins), _stream()))
        return DeviceHypergraph(k.value, l.value, net_ptr[:l.value + 1], pins[:max(npins.value, 1)])

    def dual(self, h: DeviceHypergraph) -> DeviceHypergraph:
        npins = int(h.net_ptr[-1].item())
        dptr = torch.empty(h.k + 1, dtype=torch.int64, device=h.net_ptr.device)
        dp = torch.empty(max(npins, 1), dtype=torch.int32, device=h.net_ptr.device)
        hs = h.cstruct()
        self._check(lib().vmo_dual(self.h, C.byref(hs), _ptr(dptr), _ptr(dp), _stream()))
        return DeviceHypergraph(h.l, h.k, dptr, dp, h.c, h.w)

    def components(self, h: DeviceHypergraph) -> torch.Tensor:
        lab = torch.empty(h.k, dtype=torch.int32, device=h.net_ptr.device)
        hs = h.cstruct()
        self._check(lib().vmo_components(self.h, C.byref(hs), _ptr(lab), _stream()))
        return lab

    def cut(self, h: DeviceHypergraph, part: torch.Tensor, nparts: int, noalloc: bool = False,
            part_weight: torch.Tensor | None = None):
        """Cut metrics (vmo_cut; noalloc: vmo_cut_noalloc, whose workspace is
        the library's static arena).  part_weight: an output buffer of at
        least nparts doubles (allocated here if None)."""
        pw = part_weight if part_weight is not None else torch.empty(max(nparts, 1), dtype=torch.float64,
                                                                     device=part.device)
        r = CutResult()
        hs = h.cstruct()
        fn = lib().vmo_cut_noalloc if noalloc else lib().vmo_cut
        self._check(fn(self.h, C.byref(hs), _ptr(part), C.c_int32(nparts), _ptr(pw), C.byref(r), _stream()))
        return {"lambda_minus_one": r.lambda_minus_one, "cut_net": r.cut_net, "nets_cut": r.nets_cut,
                "max_split": r.max_split, "max_split_node": r.max_split_node, "separators": bool(r.separators),
                "part_weight": pw[:nparts]}

    # ------------------------------------------------------------- bisection --
    def bisect(self, x: torch.Tensor, seed: int, t_max: int = 32):
        k = x.shape[1]
        side = torch.empty(k, dtype=torch.uint8, device=x.device)
        cen = torch.empty(8, dtype=torch.float32, device=x.device)
        it, sp = C.c_int32(), C.c_int32()
        self._check(lib().vmo_bisect(self.h, _ptr(x), C.c_int32(k), C.c_uint64(seed), C.c_int32(t_max), _ptr(side),
                                     _ptr(cen), C.byref(it), C.byref(sp), _stream()))
        return {"split": bool(sp.value), "side": side, "centres": cen.view(2, 4), "iters": it.value}

    # -------------------------------------------------------------- ordering --
    @staticmethod
    def _out(h: DeviceHypergraph, P: int, mode: int, dev):
        o = {"vperm": torch.empty(h.k, dtype=torch.int32, device=dev),
             "nperm": torch.empty(max(h.l, 1), dtype=torch.int32, device=dev) if mode == NET else None,
             "part": torch.empty(h.k, dtype=torch.int32, device=dev),
             "node_heap": torch.empty(4 * P, dtype=torch.int32, device=dev),
             "node_vptr": torch.empty(4 * P + 1, dtype=torch.int32, device=dev),
             "node_nptr": torch.empty(4 * P + 2, dtype=torch.int32, device=dev) if mode == NET else None,
             "split_cut": torch.empty(4 * P, dtype=torch.float64, device=dev),
             "n_nodes": torch.empty(1, dtype=torch.int32, device=dev)}
        s = OrderOut(*[_ptr(o[f]) for f in ("vperm", "nperm", "part", "node_heap", "node_vptr", "node_nptr",
                                            "split_cut", "n_nodes")])
        return o, s

    def order(self, h: DeviceHypergraph, x: torch.Tensor | None, P: int, seed: int, mode: int = NET,
              order: int = SBD, t_max: int = 32, lp: LayoutParams | None = None):
        dev = h.net_ptr.device
        o, s = self._out(h, P, mode, dev)
        hs = h.cstruct()
        self._check(lib().vmo_order(self.h, C.byref(hs), C.c_int(mode), C.c_int(order), _ptr(x),
                                    C.byref(lp) if lp is not None else None, C.c_int32(P), C.c_uint64(seed),
                                    C.c_int32(t_max), C.byref(s), _stream()))
        if o["nperm"] is not None:
            o["nperm"] = o["nperm"][:h.l]
        return o

    def order_border(self, h: DeviceHypergraph, o: dict, P: int, b: int, out: torch.Tensor | None = None):
        """Recursive ordering of the border (vmo_order_border): o is the dict
        order() returned for a graph-mode ordering of h; returns vperm with every
        separator block sorted by b two-bit words."""
        if out is None:
            out = torch.empty_like(o["vperm"])
        s = OrderOut(_ptr(o["vperm"]), None, _ptr(o["part"]), _ptr(o["node_heap"]), _ptr(o["node_vptr"]), None, None,
                     _ptr(o["n_nodes"]))
        hs = h.cstruct()
        self._check(lib().vmo_order_border(self.h, C.byref(hs), C.byref(s), C.c_int32(P), C.c_int32(b), _ptr(out),
                                           _stream()))
        return out

    def order_schur(self, h: DeviceHypergraph, x: torch.Tensor, o: dict, P: int, P3: int, seed: int = 0,
                    t_max: int = 32, out: torch.Tensor | None = None, mu: torch.Tensor | None = None):
        """Schur-complement recursion (vmo_order_schur): o is the dict order()
        returned for a graph-mode ordering of h at coordinates x; returns vperm
        with every separator block reordered by the BBD ordering of its induced
        graph into P3 parts (keeping the pairs of the strengthened diagonal mu
        together, if given)."""
        if out is None:
            out = torch.empty_like(o["vperm"])
        s = OrderOut(_ptr(o["vperm"]), None, _ptr(o["part"]), _ptr(o["node_heap"]), _ptr(o["node_vptr"]), None, None,
                     _ptr(o["n_nodes"]))
        hs = h.cstruct()
        self._check(lib().vmo_order_schur(self.h, C.byref(hs), _ptr(x), _ptr(mu), C.byref(s), C.c_int32(P),
                                          C.c_int32(P3), C.c_uint64(seed), C.c_int32(t_max), _ptr(out), _stream()))
        return out

    # ------------------------------------------------ strengthened diagonal --
    def match(self, m: int, n: int, rowptr: torch.Tensor, col: torch.Tensor, a: torch.Tensor | None = None,
              seed: int = 0, augment: bool = True):
        """Heavy edge matching of the bipartite graph, augmented to a maximum
        matching (vmo_match): dict with mrow, mcol, mu and size."""
        assert a is None or a.dtype == torch.float32, "a must be float32"
        dev = rowptr.device
        mrow = torch.empty(m, dtype=torch.int32, device=dev)
        mcol = torch.empty(n, dtype=torch.int32, device=dev)
        mu = torch.empty(m + n, dtype=torch.int32, device=dev)
        size = C.c_int64()
        self._check(lib().vmo_match(self.h, C.c_int32(m), C.c_int32(n), _ptr(rowptr), _ptr(col) if col.numel() else None,
                                    _ptr(a), C.c_uint32(seed), C.c_int(1 if augment else 0), _ptr(mrow), _ptr(mcol),
                                    _ptr(mu), C.byref(size), _stream()))
        return {"mrow": mrow, "mcol": mcol, "mu": mu, "size": size.value}

    def order_matched(self, h: DeviceHypergraph, x: torch.Tensor | None, mu: torch.Tensor, P: int, seed: int,
                      order: int = BBD, t_max: int = 32, lp: LayoutParams | None = None):
        """Graph-mode ordering keeping the pairs of mu together
        (vmo_order_matched)."""
        o, s = self._out(h, P, GRAPH, h.net_ptr.device)
        hs = h.cstruct()
        self._check(lib().vmo_order_matched(self.h, C.byref(hs), C.c_int(order), _ptr(x),
                                            C.byref(lp) if lp is not None else None, _ptr(mu), C.c_int32(P),
                                            C.c_uint64(seed), C.c_int32(t_max), C.byref(s), _stream()))
        return o

    def matched_perms(self, m: int, vperm: torch.Tensor, mu: torch.Tensor):
        """Row and column permutations with the matching on the diagonal."""
        rp = torch.empty(m, dtype=torch.int32, device=vperm.device)
        cp = torch.empty(m, dtype=torch.int32, device=vperm.device)
        self._check(lib().vmo_matched_perms(self.h, C.c_int32(m), _ptr(vperm), _ptr(mu), _ptr(rp), _ptr(cp),
                                            _stream()))
        return rp, cp

    def refine_kl(self, h: DeviceHypergraph, label: torch.Tensor, passes: int):
        """Kernighan-Lin passes on the bisections of a graph (vmo_refine_kl):
        label[v] = 2 g + side or -1; returns (new labels, cut reduction per
        bisection)."""
        assert label.dtype == torch.int32
        out = label.clone()
        G = C.c_int32()
        gain = torch.zeros(max(int(out.max().item()) // 2 + 1, 1), dtype=torch.int64, device=out.device)
        hs = h.cstruct()
        self._check(lib().vmo_refine_kl(self.h, C.byref(hs), _ptr(out), C.c_int32(passes), _ptr(gain), C.byref(G),
                                        _stream()))
        return out, gain[:G.value]

    def finegrain(self, m: int, n: int, rowptr: torch.Tensor, col: torch.Tensor, x: torch.Tensor):
        """Nonzero coordinates [4][nnz] from bipartite coordinates [4][m+n]."""
        nnz = int(col.numel())
        xnz = torch.empty((4, max(nnz, 1)), dtype=torch.float32, device=x.device)
        self._check(lib().vmo_finegrain(self.h, C.c_int32(m), C.c_int32(n), _ptr(rowptr),
                                        _ptr(col) if nnz else None, _ptr(x), _ptr(xnz), _stream()))
        return xnz[:, :nnz]

    def order_batch(self, jobs, t_max: int = 32, plain: bool = False):
        """jobs: list of dicts with h, x, P, seed, mode, order, job_index.  Outputs
        of all jobs share one allocation per array kind (views per job)."""
        import numpy as np
        nj = len(jobs)
        dev = jobs[0]["h"].net_ptr.device
        k = np.array([jb["h"].k for jb in jobs], np.int64)
        l = np.array([jb["h"].l for jb in jobs], np.int64)
        P = np.array([jb["P"] for jb in jobs], np.int64)
        mode = np.array([jb.get("mode", NET) for jb in jobs], np.int64)
        net = mode == NET
        nl = np.where(net, np.maximum(l, 1), 0)
        sizes = {"vperm": k, "part": k, "nperm": nl, "node_heap": 4 * P, "node_vptr": 4 * P + 1,
                 "node_nptr": np.where(net, 4 * P + 2, 0), "split_cut": 4 * P, "n_nodes": np.ones(nj, np.int64)}
        flat, offs = {}, {}
        for f, sz in sizes.items():
            dt = torch.float64 if f == "split_cut" else torch.int32
            flat[f] = torch.empty(max(int(sz.sum()), 1), dtype=dt, device=dev)
            offs[f] = np.concatenate([[0], np.cumsum(sz)[:-1]])
        arr = np.zeros(nj, dtype=_job_dtype())
        hp = [jb["h"].cptrs() for jb in jobs]
        arr["k"], arr["l"] = k, l
        arr["net_ptr"] = [a[0] for a in hp]
        arr["pins"] = [a[1] for a in hp]
        arr["w"] = [a[2] for a in hp]
        arr["c"] = [a[3] for a in hp]
        arr["mode"] = mode
        arr["order"] = [jb.get("order", SBD) for jb in jobs]
        arr["x"] = [jb["x"].data_ptr() for jb in jobs]
        arr["P"] = P
        arr["seed"] = [jb["seed"] for jb in jobs]
        arr["job_index"] = [jb.get("job_index", i) for i, jb in enumerate(jobs)]
        for f in sizes:
            ptrs = flat[f].data_ptr() + offs[f] * flat[f].element_size()
            if f in ("nperm", "node_nptr"):
                ptrs = np.where(net, ptrs, 0)
            arr["o_" + f] = ptrs
        fn = lib().vmo_order_batch_plain if plain else lib().vmo_order_batch
        self._check(fn(self.h, C.c_int32(nj), C.c_void_p(arr.ctypes.data), C.c_int32(t_max), _stream()))
        sz = {f: sizes[f].tolist() for f in sizes}
        of = {f: offs[f].tolist() for f in sizes}
        return [_BatchOut(flat, sz, of, i, bool(net[i]), int(l[i])) for i in range(nj)]

    # ---------------------------------------------------------------- layout --
    def layout(self, h: DeviceHypergraph, params: LayoutParams | None = None) -> torch.Tensor:
        params = params or layout_params()
        x = torch.empty((4, h.k), dtype=torch.float32, device=h.net_ptr.device)
        hs = h.cstruct()
        self._check(lib().vmo_layout(self.h, C.byref(hs), C.byref(params), _ptr(x), _stream()))
        return x

    def coarsen(self, h: DeviceHypergraph, seed: int, comp: int = 0, level: int = 0, match_max: int = 64):
        dev = h.net_ptr.device
        npins = int(h.net_ptr[-1].item())
        pi = torch.empty(h.k, dtype=torch.int32, device=dev)
        cptr = torch.empty(h.l + 1, dtype=torch.int64, device=dev)
        cpins = torch.empty(max(npins, 1), dtype=torch.int32, device=dev)
        cw = torch.empty(h.k, dtype=torch.float32, device=dev)
        cc = torch.empty(max(h.l, 1), dtype=torch.float32, device=dev)
        kc, lc = C.c_int32(), C.c_int32()
        hs = h.cstruct()
        self._check(lib().vmo_coarsen(self.h, C.byref(hs), C.c_uint64(seed), C.c_uint64(comp), C.c_int32(level),
                                      C.c_int32(match_max), _ptr(pi), _ptr(cptr), _ptr(cpins), _ptr(cw), _ptr(cc),
                                      C.byref(kc), C.byref(lc), _stream()))
        kc, lc = kc.value, lc.value
        return pi, DeviceHypergraph(kc, lc, cptr[:lc + 1], cpins[:max(int(cptr[lc].item()), 1)], cw[:kc], cc[:lc])

    def tree(self, x: torch.Tensor, w: torch.Tensor | None = None, leaf_cap: int = 8):
        k = x.shape[1]
        dev = x.device
        cap = 17 * k + 64
        ints = torch.empty((cap, 8), dtype=torch.int32, device=dev)
        cell2 = torch.empty((cap, 4), dtype=torch.int32, device=dev)
        flt = torch.empty((cap, 5), dtype=torch.float32, device=dev)
        order = torch.empty(k, dtype=torch.int32, device=dev)
        n = C.c_int32()
        self._check(lib().vmo_tree(self.h, _ptr(x), _ptr(w), C.c_int32(k), C.c_int32(leaf_cap), _ptr(ints),
                                   _ptr(cell2), _ptr(flt), _ptr(order), C.c_int32(cap), C.byref(n), _stream()))
        n = n.value
        return {"n": n, "ints": ints[:n], "cell2": cell2[:n], "flt": flt[:n], "order": order}

    def gradient(self, h: DeviceHypergraph, x: torch.Tensor, theta: float = 0.5, leaf_cap: int = 8):
        dev = x.device
        y = torch.empty((4, h.k), dtype=torch.float32, device=dev)
        z = torch.empty((4, max(h.l, 1)), dtype=torch.float32, device=dev)
        nint = C.c_int64()
        hs = h.cstruct()
        self._check(lib().vmo_gradient(self.h, C.byref(hs), _ptr(x), C.c_float(theta), C.c_int32(leaf_cap), _ptr(y),
                                       _ptr(z), C.byref(nint), _stream()))
        return y, z[:, :h.l], nint.value

    def layout_steps(self, h: DeviceHypergraph, x: torch.Tensor, params: LayoutParams, it0: int, iters: int,
                     alpha: float = 0.0):
        a = C.c_double(alpha)
        hs = h.cstruct()
        self._check(lib().vmo_layout_steps(self.h, C.byref(hs), C.byref(params), _ptr(x), C.c_int32(it0),
                                           C.c_int32(iters), C.byref(a), _stream()))
        return a.value


class Server:
    """Continuous-batching ordering server (vmo_serve_*).  Jobs are dicts as
    for Context.order_batch; their tensors must stay alive until done."""

    def __init__(self, budget_bytes: int = 8 << 30, max_jobs: int = 1024, t_max: int = 32, device: int = 0,
                 layout_threads: int | None = None):
        p = ServeParams()
        lib().vmo_serve_defaults(C.byref(p))
        p.device, p.budget_bytes, p.max_jobs, p.t_max = device, budget_bytes, max_jobs, t_max
        if layout_threads is not None:
            p.layout_threads = layout_threads
        h = C.c_void_p()
        st = lib().vmo_serve_create(C.byref(h), C.byref(p))
        if st != VMO_OK:
            raise VmoError(st, "vmo_serve_create failed")
        self.h = h
        self._keep = {}

    def submit(self, job: dict, lp: LayoutParams | None = None) -> int:
        h = job["h"]
        mode = job.get("mode", NET)
        o, s = Context._out(h, job["P"], mode, h.net_ptr.device)
        hs = h.cstruct()
        x = job.get("x")
        jb = Job(hs, mode, job.get("order", SBD), _ptr(x).value if x is not None else None, job["P"], job["seed"],
                 job.get("job_index", 0), s)
        t = C.c_uint64()
        torch.cuda.current_stream().synchronize()   # inputs written by torch are visible to the server's stream
        st = lib().vmo_serve_submit(self.h, C.byref(jb), C.byref(lp) if lp is not None else None, C.byref(t))
        if st != VMO_OK:
            raise VmoError(st, "vmo_serve_submit rejected the job")
        self._keep[t.value] = (job, o, s, hs, jb, lp)
        return t.value

    def poll(self, ticket: int):
        done, st, lat = C.c_int32(), C.c_int32(), C.c_double()
        r = lib().vmo_serve_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(st), C.byref(lat))
        if r != VMO_OK:
            raise VmoError(r, "unknown ticket")
        return bool(done.value), st.value, lat.value

    def wait(self, ticket: int):
        st, lat = C.c_int32(), C.c_double()
        r = lib().vmo_serve_wait(self.h, C.c_uint64(ticket), C.byref(st), C.byref(lat))
        if r != VMO_OK:
            raise VmoError(r, "unknown ticket")
        if st.value != VMO_OK:
            raise VmoError(st.value, lib().vmo_serve_error(self.h, C.c_uint64(ticket)).decode())
        job, o, *_ = self._keep.pop(ticket)
        lib().vmo_serve_forget(self.h, C.c_uint64(ticket))
        if o["nperm"] is not None:
            o["nperm"] = o["nperm"][:job["h"].l]
        return o, lat.value

    def stats(self):
        s = ServeStats()
        lib().vmo_serve_get_stats(self.h, C.byref(s))
        return {f: getattr(s, f) for f, _ in ServeStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().vmo_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
