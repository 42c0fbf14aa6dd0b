"""Torch-facing wrappers of the C ABI: hf_density, hf_l0_fof, hf_compaso, hf_find,
hf_find_batch and the hf_server request loop.

Tensors must live on the GPU the context was created on; outputs are allocated
with torch (device memory) and the work runs on torch's current stream.  The
server takes host arrays and returns host arrays.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (HfError, HfHaloSummary, HfParams, HfRequest, HfResult, HfStats, HALO_FIELDS,
                   HALO_WORDS)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_pos(pos):
    if not (isinstance(pos, torch.Tensor) and pos.is_cuda and pos.dtype == torch.float32
            and pos.dim() == 2 and pos.shape[1] == 3):
        raise ValueError("pos must be a float32 CUDA tensor of shape [n, 3]")
    return pos.contiguous()


class Context:
    """An hf_ctx on one GPU (owns the scratch arena).  budget_bytes bounds the
    device memory its arenas may hold together (0 = no bound)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.lib = _lib.load()
        self.device = int(device)
        h = ctypes.c_void_p()
        st = self.lib.hf_create(ctypes.byref(h), self.device, int(budget_bytes))
        if st:
            raise HfError(st, "hf_create failed (needs a gfx950 GPU)")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.hf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        if st:
            raise HfError(st, self.lib.hf_last_error(self.h).decode())

    def stats(self) -> dict:
        s = HfStats()
        self._raise(self.lib.hf_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in HfStats._fields_}

    # ------------------------------------------------------------ entry points
    def density(self, pos, p: HfParams):
        pos = _check_pos(pos)
        n = pos.shape[0]
        out = torch.empty(n, dtype=torch.float32, device=pos.device)
        self._raise(self.lib.hf_density(self.h, _ptr(pos), n, ctypes.byref(p), _ptr(out),
                                        _stream(pos.device)))
        return out

    def count_pairs(self, pos, p: HfParams) -> int:
        pos = _check_pos(pos)
        out = ctypes.c_int64(0)
        self._raise(self.lib.hf_count_pairs(self.h, _ptr(pos), pos.shape[0], ctypes.byref(p),
                                            ctypes.byref(out), _stream(pos.device)))
        return int(out.value)

    def l0_fof(self, pos, density, p: HfParams):
        pos = _check_pos(pos)
        n = pos.shape[0]
        density = density.contiguous()
        l0 = torch.empty(n, dtype=torch.int32, device=pos.device)
        ng = ctypes.c_int64(0)
        self._raise(self.lib.hf_l0_fof(self.h, _ptr(pos), _ptr(density), n, ctypes.byref(p),
                                       _ptr(l0), ctypes.byref(ng), _stream(pos.device)))
        return l0, ng.value

    def compaso(self, pos, density, l0_id, p: HfParams, halos_cap: int | None = None):
        pos = _check_pos(pos)
        n = pos.shape[0]
        density = density.contiguous()
        l0_id = l0_id.contiguous()
        halo_id = torch.empty(n, dtype=torch.int32, device=pos.device)
        return self._with_table(
            lambda cap, buf, nh: self.lib.hf_compaso(
                self.h, _ptr(pos), _ptr(density), _ptr(l0_id), n, ctypes.byref(p), _ptr(halo_id),
                _ptr(buf), cap, ctypes.byref(nh), _stream(pos.device)),
            halos_cap, n, pos.device, {"halo_id": halo_id})

    def find(self, pos, p: HfParams, halos_cap: int | None = None, want_density=True,
             want_l0=True):
        pos = _check_pos(pos)
        n = pos.shape[0]
        dens = torch.empty(n, dtype=torch.float32, device=pos.device) if want_density else None
        l0 = torch.empty(n, dtype=torch.int32, device=pos.device) if want_l0 else None
        halo_id = torch.empty(n, dtype=torch.int32, device=pos.device)
        return self._with_table(
            lambda cap, buf, nh: self.lib.hf_find(
                self.h, _ptr(pos), n, ctypes.byref(p), _ptr(dens), _ptr(l0), _ptr(halo_id),
                _ptr(buf), cap, ctypes.byref(nh), _stream(pos.device)),
            halos_cap, n, pos.device, {"density": dens, "l0_id": l0, "halo_id": halo_id})

    def find_grouped(self, pos, p: HfParams, halos_cap: int | None = None, want_density=True,
                     want_l0=True):
        """hf_find_grouped: hf_find plus the members in group order (Sec. 2.3.5):
        "members" (int32 [n]) holds each halo's particles (table order,
        ascending index), then the particles of no halo; "halo_start" (int64
        [n_halos + 1]) the first position of each halo's run and of the rest."""
        pos = _check_pos(pos)
        n = pos.shape[0]
        dens = torch.empty(n, dtype=torch.float32, device=pos.device) if want_density else None
        l0 = torch.empty(n, dtype=torch.int32, device=pos.device) if want_l0 else None
        halo_id = torch.empty(n, dtype=torch.int32, device=pos.device)
        members = torch.empty(max(n, 1), dtype=torch.int32, device=pos.device)
        box = {}

        def call(cap, buf, nh):
            box["start"] = torch.empty(cap + 1, dtype=torch.int64, device=pos.device)
            return self.lib.hf_find_grouped(self.h, _ptr(pos), n, ctypes.byref(p), _ptr(dens), _ptr(l0),
                                            _ptr(halo_id), _ptr(buf), cap, ctypes.byref(nh), _ptr(members),
                                            _ptr(box["start"]), _stream(pos.device))
        out = self._with_table(call, halos_cap, n, pos.device,
                               {"density": dens, "l0_id": l0, "halo_id": halo_id})
        out["members"] = members[:n]
        out["halo_start"] = box["start"][: out["n_halos"] + 1]
        return out

    def find_noalloc(self, pos, p: HfParams, halo_id, halos, density=None, l0_id=None) -> int:
        """hf_find_noalloc into caller-allocated device tensors (halo_id int32 [n],
        halos int32 [cap, HALO_WORDS], density / l0_id optional): the library's
        scratch is its static device array, so the call allocates nothing.
        Returns the halo count; raises on any error (HF_ERR_CAPACITY included)."""
        pos = _check_pos(pos)
        nh = ctypes.c_int64(0)
        st = self.lib.hf_find_noalloc(self.h, _ptr(pos), pos.shape[0], ctypes.byref(p), _ptr(density),
                                      _ptr(l0_id), _ptr(halo_id), _ptr(halos), int(halos.shape[0]),
                                      ctypes.byref(nh), _stream(pos.device))
        self._raise(st)
        return int(nh.value)

    def halo_stats(self, pos, density, halo_id, p: HfParams, n_halos: int, want_members=True):
        """hf_halo_stats: level 2 inside the L1 halos labelled by halo_id and the
        Table 1 position statistics.  Returns a dict of numpy columns (one row
        per halo, ascending id) and, with want_members, the halo-ordered member
        list and its offsets (device tensors)."""
        import numpy as np
        pos = _check_pos(pos)
        n = pos.shape[0]
        density = density.contiguous()
        halo_id = halo_id.contiguous()
        words = ctypes.sizeof(HfHaloSummary) // 4
        rows = torch.empty((max(int(n_halos), 1), words), dtype=torch.int32, device=pos.device)
        gstart = torch.empty(int(n_halos) + 1, dtype=torch.int32, device=pos.device) if want_members else None
        nmem = int((halo_id > 0).sum().item()) if want_members else 0
        members = torch.empty(max(nmem, 1), dtype=torch.int32, device=pos.device) if want_members else None
        self._raise(self.lib.hf_halo_stats(self.h, _ptr(pos), _ptr(density), _ptr(halo_id), n,
                                           ctypes.byref(p), int(n_halos), _ptr(rows), _ptr(gstart),
                                           _ptr(members), _stream(pos.device)))
        a = np.ascontiguousarray(rows[: int(n_halos)].cpu().numpy())
        f = a.view(np.float32)
        out = {"id": a[:, 0].copy(), "n": a[:, 1].copy(), "n_l2": a[:, 2].copy(),
               "l2max_nucleus": a[:, 3].copy(), "l2max_n": a[:, 4].copy(),
               "x_com": f[:, 5:8].copy(), "x_l2com": f[:, 8:11].copy(), "l2_mass": f[:, 11:16].copy(),
               "r_pct": f[:, 16:25].copy(), "vcirc_max": f[:, 25].copy(), "rvcirc_max": f[:, 26].copy()}
        if want_members:
            out["group_start"] = gstart
            out["members"] = members[:nmem]
        return out

    def find_batch(self, pos, offsets, params, halos_caps=None, n_lanes=0, want_density=True,
                   want_l0=True):
        """hf_find_batch over boxes concatenated in pos ([total, 3], device) with
        box b = rows offsets[b]:offsets[b+1]; params: one HfParams per box.
        Returns concatenated density / l0_id / halo_id (box-local labels),
        n_halos per box and the list of per-box halo tables."""
        import numpy as np
        pos = _check_pos(pos)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        nb = len(offs) - 1
        if len(params) != nb:
            raise ValueError("one HfParams per box")
        total = int(offs[-1]) if nb > 0 else 0
        if total != pos.shape[0]:
            raise ValueError("offsets[-1] must equal the number of rows of pos")
        pa = (HfParams * max(nb, 1))(*params)
        sizes = np.diff(offs)
        caps = np.maximum(sizes // 32, 1) if halos_caps is None else np.asarray(halos_caps, np.int64)
        dens = torch.empty(total, dtype=torch.float32, device=pos.device) if want_density else None
        l0 = torch.empty(total, dtype=torch.int32, device=pos.device) if want_l0 else None
        halo_id = torch.empty(total, dtype=torch.int32, device=pos.device)
        nh = np.zeros(max(nb, 1), dtype=np.int64)
        for _ in range(2):
            hoffs = np.ascontiguousarray(np.concatenate([[0], np.cumsum(caps)]), dtype=np.int64)
            buf = torch.empty((max(int(hoffs[-1]), 1), HALO_WORDS), dtype=torch.int32, device=pos.device)
            st = self.lib.hf_find_batch(self.h, nb, offs.ctypes.data, _ptr(pos), ctypes.byref(pa),
                                        _ptr(dens), _ptr(l0), _ptr(halo_id), _ptr(buf),
                                        hoffs.ctypes.data, nh.ctypes.data, int(n_lanes),
                                        _stream(pos.device))
            if st == _lib.HF_ERR_CAPACITY:
                caps = np.maximum(caps, nh[:nb])
                continue
            self._raise(st)
            tables = [buf[hoffs[b]: hoffs[b] + nh[b]] for b in range(nb)]
            return {"density": dens, "l0_id": l0, "halo_id": halo_id, "n_halos": nh[:nb].copy(),
                    "halos": tables}
        raise HfError(_lib.HF_ERR_CAPACITY, "halo table capacity retry failed")

    def set_radius_search(self, mode: str):
        """hf_set_option(HF_OPT_RADIUS_SEARCH): "histogram" (default) or "bins"
        (the radial bins of Sec. 2.3.4); the results are the same."""
        value = {"histogram": _lib.HF_RADIUS_HISTOGRAM, "bins": _lib.HF_RADIUS_BINS}[mode]
        self._raise(self.lib.hf_set_option(self.h, _lib.HF_OPT_RADIUS_SEARCH, value))

    def radius_search(self) -> str:
        v = ctypes.c_int64(-1)
        self._raise(self.lib.hf_get_option(self.h, _lib.HF_OPT_RADIUS_SEARCH, ctypes.byref(v)))
        return "bins" if v.value == _lib.HF_RADIUS_BINS else "histogram"

    def tune_batch(self, pos, offsets, params, max_groups=4, reps=2, table_path=None):
        """hf_tune_batch: times hf_find_batch on these boxes with 1..max_groups
        fused groups and records the fastest count for this batch shape (in the
        context, and in table_path when given).  Returns (best_groups, best_ms,
        results as find_batch returns them)."""
        import numpy as np
        first = self.find_batch(pos, offsets, params, n_lanes=1)
        pos = _check_pos(pos)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        nb = len(offs) - 1
        total = int(offs[-1])
        pa = (HfParams * max(nb, 1))(*params)
        caps = np.maximum(first["n_halos"], 1)
        hoffs = np.ascontiguousarray(np.concatenate([[0], np.cumsum(caps)]), dtype=np.int64)
        buf = torch.empty((int(hoffs[-1]), HALO_WORDS), dtype=torch.int32, device=pos.device)
        dens = torch.empty(total, dtype=torch.float32, device=pos.device)
        l0 = torch.empty(total, dtype=torch.int32, device=pos.device)
        halo_id = torch.empty(total, dtype=torch.int32, device=pos.device)
        nh = np.zeros(max(nb, 1), dtype=np.int64)
        best = ctypes.c_int32(0)
        ms = ctypes.c_float(0.0)
        path = table_path.encode() if table_path else None
        self._raise(self.lib.hf_tune_batch(self.h, nb, offs.ctypes.data, _ptr(pos), ctypes.byref(pa), _ptr(dens),
                                           _ptr(l0), _ptr(halo_id), _ptr(buf), hoffs.ctypes.data,
                                           nh.ctypes.data, int(max_groups), int(reps), path,
                                           ctypes.byref(best), ctypes.byref(ms), _stream(pos.device)))
        tables = [buf[hoffs[b]: hoffs[b] + nh[b]] for b in range(nb)]
        return best.value, ms.value, {"density": dens, "l0_id": l0, "halo_id": halo_id,
                                      "n_halos": nh[:nb].copy(), "halos": tables}

    def load_tuning(self, table_path):
        """hf_load_tuning: take a tuning table's lines for this device; returns
        the number of lines taken."""
        k = ctypes.c_int32(0)
        self._raise(self.lib.hf_load_tuning(self.h, table_path.encode(), ctypes.byref(k)))
        return k.value

    def batch_groups(self, n_boxes, total, n_lanes=0):
        """hf_batch_groups: the fused group count hf_find_batch would use."""
        g = ctypes.c_int32(0)
        self._raise(self.lib.hf_batch_groups(self.h, int(n_boxes), int(total), int(n_lanes), ctypes.byref(g)))
        return g.value

    def _with_table(self, call, cap, n, device, outs):
        cap = max(1, n // 32) if cap is None else int(cap)
        for _ in range(2):
            buf = torch.empty((max(cap, 1), HALO_WORDS), dtype=torch.int32, device=device)
            nh = ctypes.c_int64(0)
            st = call(cap, buf, nh)
            if st == _lib.HF_ERR_CAPACITY:
                cap = int(nh.value)
                continue
            self._raise(st)
            outs["n_halos"] = int(nh.value)
            outs["halos"] = buf[: nh.value]
            return outs
        raise HfError(_lib.HF_ERR_CAPACITY, "halo table capacity retry failed")


class Server:
    """An hf_server: requests (host positions) run on `slots` pipelines at once
    within an HBM budget; results come back in page-locked host tensors."""

    def __init__(self, device: int = 0, slots: int = 4, budget_bytes: int = 64 << 30):
        self.lib = _lib.load()
        self.device = int(device)
        h = ctypes.c_void_p()
        st = self.lib.hf_server_create(ctypes.byref(h), self.device, int(slots), int(budget_bytes))
        if st:
            raise HfError(st, "hf_server_create failed")
        self.h = h
        self._live = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.hf_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def now(self) -> float:
        return float(self.lib.hf_server_now(self.h))

    def held_bytes(self) -> int:
        return int(self.lib.hf_server_held_bytes(self.h))

    @staticmethod
    def pinned_positions(pos) -> torch.Tensor:
        """A page-locked float32 [n, 3] copy of pos (numpy or torch)."""
        t = torch.as_tensor(pos, dtype=torch.float32).reshape(-1, 3)
        out = torch.empty(t.shape, dtype=torch.float32, pin_memory=True)
        out.copy_(t)
        return out

    def submit(self, pos, p: HfParams, halos_cap: int | None = None, want_density=False,
               want_l0=False) -> int:
        """Queue one box; pos is a host float32 [n, 3] array (page-locked when it
        comes from pinned_positions, which makes the device copy asynchronous)."""
        if isinstance(pos, torch.Tensor) and pos.is_pinned() and pos.dtype == torch.float32:
            pos_h = pos.contiguous()
        else:
            pos_h = self.pinned_positions(pos)
        n = pos_h.shape[0]
        cap = max(1, n // 32) if halos_cap is None else int(halos_cap)
        bufs = {"pos": pos_h,
                "halo_id": torch.empty(n, dtype=torch.int32, pin_memory=True),
                "halos": torch.empty((max(cap, 1), HALO_WORDS), dtype=torch.int32, pin_memory=True),
                "density": torch.empty(n, dtype=torch.float32, pin_memory=True) if want_density else None,
                "l0_id": torch.empty(n, dtype=torch.int32, pin_memory=True) if want_l0 else None}
        req = HfRequest()
        req.pos = pos_h.data_ptr() if n else None
        req.n = n
        req.params = p
        req.density = bufs["density"].data_ptr() if want_density and n else None
        req.l0_id = bufs["l0_id"].data_ptr() if want_l0 and n else None
        req.halo_id = bufs["halo_id"].data_ptr() if n else None
        req.halos = bufs["halos"].data_ptr()
        req.halos_cap = cap
        ticket = ctypes.c_int64(0)
        st = self.lib.hf_server_submit(self.h, ctypes.byref(req), ctypes.byref(ticket))
        if st:
            raise HfError(st, self.lib.hf_server_last_error(self.h).decode())
        self._live[ticket.value] = bufs
        return ticket.value

    def wait(self, ticket: int, check: bool = True) -> dict:
        res = HfResult()
        st = self.lib.hf_server_wait(self.h, int(ticket), ctypes.byref(res))
        if st:
            raise HfError(st, self.lib.hf_server_last_error(self.h).decode())
        bufs = self._live.pop(ticket)
        if check and res.status:
            raise HfError(res.status, res.error.decode())
        nh = int(res.n_halos)
        return {"status": int(res.status), "error": res.error.decode(), "slot": int(res.slot),
                "n_halos": nh, "halo_id": bufs["halo_id"], "density": bufs["density"],
                "l0_id": bufs["l0_id"], "halos": bufs["halos"][:nh] if res.status == 0 else None,
                "t_submit": res.t_submit, "t_start": res.t_start, "t_done": res.t_done,
                "ms_gpu": float(res.ms_gpu)}


def halo_table(rows: torch.Tensor) -> dict:
    """Split an [n_halos, 10] int32 table (hf_halo rows) into named numpy columns."""
    import numpy as np
    a = rows.cpu().numpy()
    out = {}
    for k, name in enumerate(HALO_FIELDS):
        col = a[:, k]
        out[name] = col.view(np.float32) if name in ("x", "y", "z", "r", "mass") else col.copy()
    return out
