"""Torch-facing wrappers of the C ABI: hf_density, hf_l0_fof, hf_compaso, hf_find.

Tensors must live on the GPU the context was created on; outputs are allocated
with torch (device memory) and the work runs on torch's current stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import HfError, HfParams, HfStats, HALO_FIELDS, HALO_WORDS


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
    """An hf_ctx on one GPU (owns the scratch arena)."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        self.device = int(device)
        h = ctypes.c_void_p()
        st = self.lib.hf_create(ctypes.byref(h), self.device)
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


def halo_table(rows: torch.Tensor) -> dict:
    """Split an [n_halos, 10] int32 table (hf_halo rows) into named numpy columns."""
    import numpy as np
    a = rows.cpu().numpy()
    out = {}
    for k, name in enumerate(HALO_FIELDS):
        col = a[:, k]
        out[name] = col.view(np.float32) if name in ("x", "y", "z", "r", "mass") else col.copy()
    return out
