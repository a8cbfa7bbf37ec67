"""VOctree container: the octree built on the host by the C ABI, the leaf
payload packed on the device by the library, the temporal tables, all as
torch device tensors (torch only holds the memory)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib

_TORCH_DTYPE = {_lib.F32: torch.float32, _lib.F16: torch.float16, _lib.BF16: torch.bfloat16}


def build_child_table(depth: int, leaf_ijk: np.ndarray):
    """Host octree over the leaf cells: (child [n_nodes,8] int32, slot_of_input [N] int64)."""
    ijk = np.ascontiguousarray(leaf_ijk, dtype=np.int32).reshape(-1, 3)
    n_nodes = _lib.neuvv_build_voctree(depth, ijk)
    child = np.empty((n_nodes, 8), np.int32)
    slots = np.empty(ijk.shape[0], np.int64)
    _lib.neuvv_build_voctree(depth, ijk, child, n_nodes, slots)
    return child, slots


@dataclass
class VOctree:
    depth: int
    K: int
    C: int
    T: int
    dtype: int
    n_leaves: int
    child: torch.Tensor          # [n_nodes, 8] int32
    hh: torch.Tensor             # packed colour coefficients (storage dtype)
    wsig: torch.Tensor           # packed density weights (storage dtype)
    basis: torch.Tensor          # [T, C] float32
    gamma: torch.Tensor          # [T] float32
    slot_of_input: torch.Tensor  # [N] int64, device

    @classmethod
    def build(cls, depth: int, leaf_ijk, hh, wsig, basis, gamma, dtype: int = _lib.F32,
              device: str = "cuda", stream=None) -> "VOctree":
        """leaf_ijk [N,3]; hh [N,3,K] and wsig [N,C] float32 per input leaf; basis [T,C]; gamma [T]."""
        child, slots = build_child_table(depth, leaf_ijk)
        hh = np.ascontiguousarray(hh, np.float32)
        wsig = np.ascontiguousarray(wsig, np.float32)
        N, _, K = hh.shape
        C = wsig.shape[1]
        dev = torch.device(device)
        t = cls(depth, K, C, int(np.asarray(basis).shape[0]), dtype, N,
                torch.from_numpy(child).to(dev), None, None,
                torch.from_numpy(np.ascontiguousarray(basis, np.float32)).to(dev),
                torch.from_numpy(np.ascontiguousarray(gamma, np.float32)).to(dev),
                torch.from_numpy(slots).to(dev))
        t.set_payload(torch.from_numpy(hh).to(dev), torch.from_numpy(wsig).to(dev), stream=stream)
        return t

    def payload_elems(self, dtype: Optional[int] = None):
        return _lib.neuvv_payload_words(self.K, self.C, self.dtype if dtype is None else dtype, self.n_leaves)

    def set_payload(self, hh_in: torch.Tensor, wsig_in: torch.Tensor, stream=None):
        """(Re)packs float32 coefficients given per input leaf ([N,3,K], [N,C], device)."""
        a, b = self.payload_elems()
        td = _TORCH_DTYPE[self.dtype]
        dev = self.child.device
        if self.hh is None or self.hh.numel() != a:
            self.hh = torch.empty(a, dtype=td, device=dev)
            self.wsig = torch.empty(b, dtype=td, device=dev)
        _lib.neuvv_pack_leaves(self.K, self.C, self.dtype, self.n_leaves, hh_in.contiguous().float(),
                               wsig_in.contiguous().float(), self.slot_of_input, self.hh, self.wsig, stream)

    def struct(self) -> _lib.neuvv_tree:
        s = _lib.neuvv_tree()
        s.depth, s.K, s.C, s.dtype = self.depth, self.K, self.C, self.dtype
        s.n_nodes, s.n_leaves = int(self.child.shape[0]), self.n_leaves
        s.child, s.hh, s.wsig = self.child.data_ptr(), self.hh.data_ptr(), self.wsig.data_ptr()
        s.T, s.basis, s.gamma = self.T, self.basis.data_ptr(), self.gamma.data_ptr()
        return s

    def zero_grads(self):
        """Float32 gradient buffers in the float32 payload layout, and [T,C] for the basis."""
        a, b = self.payload_elems(_lib.F32)
        dev = self.child.device
        return (torch.zeros(a, dtype=torch.float32, device=dev), torch.zeros(b, dtype=torch.float32, device=dev),
                torch.zeros(self.T, self.C, dtype=torch.float32, device=dev))

    def unpack_f32(self, packed_hh: torch.Tensor, packed_wsig: torch.Tensor):
        """Float32 packed arrays -> per input leaf [N,3,K] and [N,C] (layout permutation only)."""
        N, K, C = self.n_leaves, self.K, self.C
        gh = -(-3 * K // 4)
        gw = -(-C // 4)
        hh = packed_hh.view(gh, N, 4).permute(1, 0, 2).reshape(N, gh * 4)[:, :3 * K].reshape(N, 3, K)
        ws = packed_wsig.view(gw, N, 4).permute(1, 0, 2).reshape(N, gw * 4)[:, :C]
        return hh[self.slot_of_input], ws[self.slot_of_input]
