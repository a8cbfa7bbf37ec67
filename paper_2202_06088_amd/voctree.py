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


def build_node_table(depth: int, leaf_ijk: np.ndarray, with_box: bool = False):
    """Host octree over the leaf cells, two levels per node row:
    (nodes [n_nodes,4] int32, slot_of_input [N] int64[, box [6]])."""
    ijk = np.ascontiguousarray(leaf_ijk, dtype=np.int32).reshape(-1, 3)
    n_nodes = _lib.neuvv_build_voctree(depth, ijk)
    nodes = np.empty((n_nodes, 4), np.int32)
    slots = np.empty(ijk.shape[0], np.int64)
    box = np.zeros(6, np.int32)
    _lib.neuvv_build_voctree(depth, ijk, nodes, n_nodes, slots, box)
    return (nodes, slots, box) if with_box else (nodes, slots)


@dataclass
class VOctree:
    depth: int
    K: int
    C: int
    T: int
    dtype: int
    n_leaves: int
    nodes: torch.Tensor          # [n_nodes, 4] int32 node rows (mask lo, mask hi, first child, 0)
    hh: torch.Tensor             # packed colour coefficients (storage dtype)
    wsig: torch.Tensor           # packed density weights (storage dtype)
    basis: torch.Tensor          # [T, C] float32
    gamma: torch.Tensor          # [T] float32
    slot_of_input: torch.Tensor  # [N] int64, device
    box: tuple = (0, 0, 0, 0, 0, 0)  # occupied-cell bounds (lo xyz, hi xyz exclusive)
    layout: int = _lib.LAYOUT_LEAF_ROWS

    @classmethod
    def build(cls, depth: int, leaf_ijk, hh, wsig, basis, gamma, dtype: int = _lib.F32,
              device: str = "cuda", stream=None, layout: int = _lib.LAYOUT_LEAF_ROWS) -> "VOctree":
        """leaf_ijk [N,3]; hh [N,3,K] and wsig [N,C] float32 per input leaf; basis [T,C]; gamma [T]."""
        nodes, slots, box = build_node_table(depth, leaf_ijk, with_box=True)
        hh = np.ascontiguousarray(hh, np.float32)
        wsig = np.ascontiguousarray(wsig, np.float32)
        N, _, K = hh.shape
        C = wsig.shape[1]
        dev = torch.device(device)
        t = cls(depth, K, C, int(np.asarray(basis).shape[0]), dtype, N,
                torch.from_numpy(nodes).to(dev), None, None,
                torch.from_numpy(np.ascontiguousarray(basis, np.float32)).to(dev),
                torch.from_numpy(np.ascontiguousarray(gamma, np.float32)).to(dev),
                torch.from_numpy(slots).to(dev), tuple(int(v) for v in box), layout)
        t.set_payload(torch.from_numpy(hh).to(dev), torch.from_numpy(wsig).to(dev), stream=stream)
        return t

    def payload_elems(self, dtype: Optional[int] = None):
        return _lib.neuvv_payload_words(self.K, self.C, self.dtype if dtype is None else dtype, self.n_leaves)

    def set_payload(self, hh_in: torch.Tensor, wsig_in: torch.Tensor, stream=None):
        """(Re)packs float32 coefficients given per input leaf ([N,3,K], [N,C], device)."""
        a, b = self.payload_elems()
        td = _TORCH_DTYPE[self.dtype]
        dev = self.nodes.device
        if self.hh is None or self.hh.numel() != a:
            self.hh = torch.empty(a, dtype=td, device=dev)
            self.wsig = torch.empty(b, dtype=td, device=dev)
        _lib.neuvv_pack_leaves(self.K, self.C, self.dtype, self.layout, self.n_leaves, hh_in.contiguous().float(),
                               wsig_in.contiguous().float(), self.slot_of_input, self.hh, self.wsig, stream)

    def struct(self) -> _lib.neuvv_tree:
        s = _lib.neuvv_tree()
        s.depth, s.K, s.C, s.dtype = self.depth, self.K, self.C, self.dtype
        s.n_nodes, s.n_leaves = int(self.nodes.shape[0]), self.n_leaves
        s.nodes, s.hh, s.wsig = self.nodes.data_ptr(), self.hh.data_ptr(), self.wsig.data_ptr()
        s.T, s.basis, s.gamma = self.T, self.basis.data_ptr(), self.gamma.data_ptr()
        for i in range(6):
            s.box[i] = self.box[i]
        s.layout = self.layout
        return s

    @property
    def grad_row(self) -> int:
        return _lib.neuvv_grad_row_elems(self.K, self.C)

    def zero_grads(self):
        """Zeroed float32 gradient buffers: leaf rows [N, ROW] and the basis [T, C]."""
        dev = self.nodes.device
        return (torch.zeros(self.n_leaves, self.grad_row, dtype=torch.float32, device=dev),
                torch.zeros(self.T, self.C, dtype=torch.float32, device=dev))

    def unpack_grad(self, grad_leaf: torch.Tensor):
        """Leaf gradient rows (slot order) -> per input leaf d/dhh [N,3,K] and d/dwsig [N,C]."""
        K, C = self.K, self.C
        rows = grad_leaf.view(self.n_leaves, self.grad_row)[self.slot_of_input]
        return rows[:, :3 * K].reshape(-1, 3, K), rows[:, 3 * K:3 * K + C]

    def rows_to_payload_f32(self, grad_leaf: torch.Tensor):
        """Leaf gradient rows -> the float32 payload layout of hh and wsig (a rearrangement
        only), for an element-wise optimizer step on float32 payload tensors."""
        N, K, C = self.n_leaves, self.K, self.C
        rows = grad_leaf.view(N, self.grad_row)
        gh, gw = -(-3 * K // 4), -(-C // 4)
        hh = torch.zeros(N, gh * 4, device=rows.device)
        hh[:, :3 * K] = rows[:, :3 * K]
        ws = torch.zeros(N, gw * 4, device=rows.device)
        ws[:, :C] = rows[:, 3 * K:3 * K + C]
        if self.layout == _lib.LAYOUT_LEAF_ROWS:
            return hh.reshape(-1).contiguous(), ws.reshape(-1).contiguous()
        return (hh.view(N, gh, 4).permute(1, 0, 2).reshape(-1).contiguous(),
                ws.view(N, gw, 4).permute(1, 0, 2).reshape(-1).contiguous())
