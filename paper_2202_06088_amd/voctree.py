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
    Cg: int = 0                  # per-point hyperangle weights per leaf (Eq. 6); 0 = global gamma table
    wgam: Optional[torch.Tensor] = None     # packed hyperangle weights (storage dtype)
    basis_g: Optional[torch.Tensor] = None  # [T, Cg] float32 hyperangle basis
    edit: Optional[torch.Tensor] = None     # [N, 8] float32 appearance-edit rows (slot order), or None
    density: int = _lib.DENSITY_SOFTPLUS    # activation of Eq. 5 (softplus, or ReLU as Eq. 5 prints it)
    dir: Optional[torch.Tensor] = None      # brick directory of the node table (neuvv_build_directory)

    @classmethod
    def build(cls, depth: int, leaf_ijk, hh, wsig, basis, gamma, dtype: int = _lib.F32,
              device: str = "cuda", stream=None, layout: int = _lib.LAYOUT_LEAF_ROWS, wgam=None,
              basis_g=None, density: int = _lib.DENSITY_SOFTPLUS) -> "VOctree":
        """leaf_ijk [N,3]; hh [N,3,K] and wsig [N,C] float32 per input leaf; basis [T,C]; gamma [T]
        (or None with the per-point form); wgam [N,Cg] and basis_g [T,Cg] for the per-point
        hyperangle of Eq. 6."""
        nodes, slots, box = build_node_table(depth, leaf_ijk, with_box=True)
        hh = np.ascontiguousarray(hh, np.float32)
        wsig = np.ascontiguousarray(wsig, np.float32)
        N, _, K = hh.shape
        C = wsig.shape[1]
        dev = torch.device(device)
        T = int(np.asarray(basis).shape[0])
        if gamma is None:
            if wgam is None:
                raise ValueError("gamma is required without per-point hyperangle weights")
            gamma = np.zeros(T, np.float32)
        t = cls(depth, K, C, T, dtype, N,
                torch.from_numpy(nodes).to(dev), None, None,
                torch.from_numpy(np.ascontiguousarray(basis, np.float32)).to(dev),
                torch.from_numpy(np.ascontiguousarray(gamma, np.float32)).to(dev),
                torch.from_numpy(slots).to(dev), tuple(int(v) for v in box), layout)
        t.density = int(density)
        t.build_directory(stream)
        wg = None
        if wgam is not None:
            wgam = np.ascontiguousarray(wgam, np.float32)
            t.Cg = int(wgam.shape[1])
            t.basis_g = torch.from_numpy(np.ascontiguousarray(basis_g, np.float32)).to(dev)
            wg = torch.from_numpy(wgam).to(dev)
        t.set_payload(torch.from_numpy(hh).to(dev), torch.from_numpy(wsig).to(dev), wg, stream=stream)
        return t

    def build_directory(self, stream=None):
        """(Re)builds the brick directory the walk reads, from the device node table."""
        n = _lib.neuvv_directory_entries(self.depth)
        if self.dir is None or self.dir.numel() != n:
            self.dir = torch.empty(n, dtype=torch.int32, device=self.nodes.device)
        _lib.neuvv_build_directory(self.depth, int(self.nodes.shape[0]), self.nodes, self.dir, n, stream)

    def payload_elems(self, dtype: Optional[int] = None):
        return _lib.neuvv_payload_words(self.K, self.C, self.dtype if dtype is None else dtype, self.n_leaves)

    def set_payload(self, hh_in: torch.Tensor, wsig_in: torch.Tensor, wgam_in: Optional[torch.Tensor] = None,
                    stream=None):
        """(Re)packs float32 coefficients given per input leaf ([N,3,K], [N,C], and [N,Cg] for
        the per-point form; device)."""
        a, b = self.payload_elems()
        td = _TORCH_DTYPE[self.dtype]
        dev = self.nodes.device
        if self.hh is None or self.hh.numel() != a:
            self.hh = torch.empty(a, dtype=td, device=dev)
            self.wsig = torch.empty(b, dtype=td, device=dev)
        _lib.neuvv_pack_leaves(self.K, self.C, self.dtype, self.layout, self.n_leaves, hh_in.contiguous().float(),
                               wsig_in.contiguous().float(), self.slot_of_input, self.hh, self.wsig, stream)
        if self.Cg > 0:
            if wgam_in is None:
                raise ValueError("this tree needs its per-point hyperangle weights")
            _, g = _lib.neuvv_payload_words(self.K, self.Cg, self.dtype, self.n_leaves)
            if self.wgam is None or self.wgam.numel() != g:
                self.wgam = torch.empty(g, dtype=td, device=dev)
            _lib.neuvv_pack_rows(self.Cg, self.dtype, self.layout, self.n_leaves, wgam_in.contiguous().float(),
                                 self.slot_of_input, self.wgam, stream)

    def struct(self) -> _lib.neuvv_tree:
        s = _lib.neuvv_tree()
        s.depth, s.K, s.C, s.dtype = self.depth, self.K, self.C, self.dtype
        s.n_nodes, s.n_leaves = int(self.nodes.shape[0]), self.n_leaves
        s.nodes, s.hh, s.wsig = self.nodes.data_ptr(), self.hh.data_ptr(), self.wsig.data_ptr()
        s.T, s.basis, s.gamma = self.T, self.basis.data_ptr(), self.gamma.data_ptr()
        for i in range(6):
            s.box[i] = self.box[i]
        s.layout = self.layout
        s.Cg = self.Cg
        if self.Cg > 0:
            s.wgam, s.basis_g = self.wgam.data_ptr(), self.basis_g.data_ptr()
        s.edit = None if self.edit is None else self.edit.data_ptr()
        s.density = self.density
        s.dir = self.dir.data_ptr()
        return s

    def enable_edits(self):
        """Attaches an appearance-edit table (Sec. 5.2) with every edit inactive (first frame
        +inf, target density -1 = keep); neuvv_paint fills it."""
        e = torch.zeros(self.n_leaves, 8, dtype=torch.float32, device=self.nodes.device)
        e[:, 3] = -1.0
        e[:, 4] = float("inf")
        self.edit = e
        return e

    def edits_per_input(self) -> torch.Tensor:
        """The edit table as [N, 5] (rgb, sigma_d, t_d) per input leaf."""
        return self.edit[self.slot_of_input][:, :5]

    @property
    def grad_row(self) -> int:
        return _lib.neuvv_grad_row_elems(self.K, self.C, self.Cg)

    def zero_grads(self):
        """Zeroed float32 gradient buffers: leaf rows [N, ROW] and the basis [T, C] (and the
        hyperangle basis [T, Cg] for the per-point form)."""
        dev = self.nodes.device
        g = (torch.zeros(self.n_leaves, self.grad_row, dtype=torch.float32, device=dev),
             torch.zeros(self.T, self.C, dtype=torch.float32, device=dev))
        if self.Cg > 0:
            g = g + (torch.zeros(self.T, self.Cg, dtype=torch.float32, device=dev),)
        return g

    def unpack_grad(self, grad_leaf: torch.Tensor):
        """Leaf gradient rows (slot order) -> per input leaf d/dhh [N,3,K] and d/dwsig [N,C]
        (and d/dwgam [N,Cg] for the per-point form)."""
        K, C, G = self.K, self.C, self.Cg
        rows = grad_leaf.view(self.n_leaves, self.grad_row)[self.slot_of_input]
        out = (rows[:, :3 * K].reshape(-1, 3, K), rows[:, 3 * K:3 * K + C])
        if G > 0:
            out = out + (rows[:, 3 * K + C:3 * K + C + G],)
        return out

    def rows_to_payload_f32(self, grad_leaf: torch.Tensor):
        """Leaf gradient rows -> the float32 payload layout of hh and wsig (and wgam), a
        rearrangement only, for an element-wise optimizer step on float32 payload tensors."""
        N, K, C, G = self.n_leaves, self.K, self.C, self.Cg
        rows = grad_leaf.view(N, self.grad_row)
        parts = [(0, 3 * K), (3 * K, C)] + ([(3 * K + C, G)] if G > 0 else [])
        out = []
        for start, R in parts:
            ng = -(-R // 4)
            a = torch.zeros(N, ng * 4, device=rows.device)
            a[:, :R] = rows[:, start:start + R]
            if self.layout == _lib.LAYOUT_LEAF_ROWS:
                out.append(a.reshape(-1).contiguous())
            else:
                out.append(a.view(N, ng, 4).permute(1, 0, 2).reshape(-1).contiguous())
        return tuple(out)
