"""Torch-side conveniences over the C ABI: device buffers as raw byte tensors.

PyTorch only provides device memory and streams here; the sort itself is the
library's.  Buffers are uint8 tensors holding the raw bytes of the keys
(uint32 / uint64 / int64 / 16-byte rows) and the uint32 payload.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B


def to_device(a: np.ndarray, device: str = "cuda") -> torch.Tensor:
    raw = np.ascontiguousarray(a).reshape(-1).view(np.uint8)
    t = torch.empty(raw.shape[0], dtype=torch.uint8, device=device)
    if raw.shape[0]:
        t.copy_(torch.from_numpy(raw))
    return t


def empty_device(nbytes: int, device: str = "cuda") -> torch.Tensor:
    # at least 256 bytes so data_ptr() is a real, aligned allocation
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def to_host(t: torch.Tensor, dtype, shape) -> np.ndarray:
    dtype = np.dtype(dtype)
    count = int(np.prod(shape)) * dtype.itemsize
    return t[:count].cpu().numpy().view(dtype).reshape(shape)


def sort_keys(desc: B.KeyDesc, keys: torch.Tensor, n: int, out: torch.Tensor | None = None,
              tmp: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Sorts n keys held in `keys` (raw bytes); returns the output buffer."""
    out = torch.empty_like(keys) if out is None else out
    need = B.rs_temp_bytes(desc, n, False)
    tmp = empty_device(need, keys.device) if tmp is None else tmp
    B.rs_sort_keys(desc, keys, out, n, tmp, tmp.numel(), stream)
    return out


def sort_pairs(desc: B.KeyDesc, keys: torch.Tensor, vals: torch.Tensor, n: int,
               keys_out: torch.Tensor | None = None, vals_out: torch.Tensor | None = None,
               tmp: torch.Tensor | None = None, stream=None):
    """Stable sort of n (key, uint32) pairs; returns (keys_out, vals_out)."""
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    need = B.rs_temp_bytes(desc, n, True)
    tmp = empty_device(need, keys.device) if tmp is None else tmp
    B.rs_sort_pairs(desc, keys, keys_out, vals, vals_out, n, tmp, tmp.numel(), stream)
    return keys_out, vals_out


def sort_batched(desc: B.KeyDesc, keys: torch.Tensor, vals: torch.Tensor | None, offsets: torch.Tensor,
                 nseg: int, total: int, keys_out: torch.Tensor | None = None,
                 vals_out: torch.Tensor | None = None, tmp: torch.Tensor | None = None, stream=None):
    """Sorts nseg arrays (device uint64 offsets [nseg + 1]); returns outputs."""
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    need = B.rs_batched_temp_bytes(desc, total, nseg, vals is not None)
    tmp = empty_device(need, keys.device) if tmp is None else tmp
    B.rs_sort_batched(desc, keys, keys_out, vals, vals_out, offsets, nseg, total, tmp, tmp.numel(), stream)
    return keys_out, vals_out
