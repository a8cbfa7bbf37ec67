"""ctypes binding of libneuvv.so: the C ABI of include/neuvv.h, same names,
argument marshalling only. Device buffers are torch tensors (data_ptr()),
streams are torch streams (cuda_stream). There is no fallback: if the library
is not built, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libneuvv.so")

NEUVV_OK = 0
F32, F16, BF16 = 0, 1, 2
LAYOUT_VEC_SOA, LAYOUT_LEAF_ROWS = 0, 1
DENSITY_SOFTPLUS, DENSITY_RELU = 0, 1


class NeuvvError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


class neuvv_tree(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("K", ctypes.c_int32), ("C", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("n_nodes", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("nodes", ctypes.c_void_p), ("hh", ctypes.c_void_p), ("wsig", ctypes.c_void_p),
                ("T", ctypes.c_int32), ("box", ctypes.c_int32 * 6), ("layout", ctypes.c_int32),
                ("basis", ctypes.c_void_p), ("gamma", ctypes.c_void_p), ("Cg", ctypes.c_int32),
                ("wgam", ctypes.c_void_p), ("basis_g", ctypes.c_void_p), ("edit", ctypes.c_void_p),
                ("density", ctypes.c_int32), ("dir", ctypes.c_void_p)]


class neuvv_instance(ctypes.Structure):
    _fields_ = [("rot", ctypes.c_float * 9), ("trans", ctypes.c_float * 3), ("scale", ctypes.c_float),
                ("time_offset", ctypes.c_float), ("time_wrap", ctypes.c_int32)]


class neuvv_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("c2w", ctypes.c_float * 12)]


class neuvv_light(ctypes.Structure):
    _fields_ = [("camera", neuvv_camera), ("ground_z", ctypes.c_float), ("ground_rgb", ctypes.c_float * 3),
                ("background_rgb", ctypes.c_float * 3), ("shadow_strength", ctypes.c_float),
                ("falloff_r0", ctypes.c_float)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F = ctypes.c_float

_SIGNATURES = {
    "neuvv_build_voctree": [_I32, _I64, _P, _P, _I64, _P, _P, _P],
    "neuvv_payload_words": [_I32, _I32, _I32, _I64, _P, _P],
    "neuvv_build_directory": [_I32, _I64, _P, _P, _I64, _P],
    "neuvv_pack_leaves": [_I32, _I32, _I32, _I32, _I64, _P, _P, _P, _P, _P, _P],
    "neuvv_render": [ctypes.POINTER(neuvv_tree), ctypes.POINTER(neuvv_instance), _I64, _P, _P, _P, _F, _I32, _F,
                     _P, _P, _P, _P, _P],
    "neuvv_render_noalloc": [ctypes.POINTER(neuvv_tree), ctypes.POINTER(neuvv_instance), _I64, _P, _P, _P, _F, _I32,
                             _F, _P, _P, _P, _P, _P],
    "neuvv_render_backward": [ctypes.POINTER(neuvv_tree), ctypes.POINTER(neuvv_instance), _I64, _P, _P, _P, _F,
                              _I32, _F, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "neuvv_render_trace": [ctypes.POINTER(neuvv_tree), ctypes.POINTER(neuvv_instance), _I64, _P, _P, _P, _F, _I32,
                           _F, _P, _P, _P, _P, _P, _I64, _P],
    "neuvv_render_backward_trace": [ctypes.POINTER(neuvv_tree), ctypes.POINTER(neuvv_instance), _I64, _P, _P, _P,
                                    _F, _I32, _F, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _P],
    "neuvv_grad_row_elems": [_I32, _I32, _I32],
    "neuvv_pack_rows": [_I32, _I32, _I32, _I64, _P, _P, _P, _P],
    "neuvv_blur": [_I32, _I32, _P, _F, _P, _P],
    "neuvv_find_terminal_leaves": [ctypes.POINTER(neuvv_tree), ctypes.POINTER(neuvv_instance), _I64, _P, _P, _P, _F,
                                   _I32, _F, _P, _P],
    "neuvv_paint": [_I64, _P, _P, _F, _F, _I64, _P, _P],
    "neuvv_render_multi": [_I32, _P, _P, _I64, _P, _P, _P, _F, _I32, _F, _P, _P, _P, _P, _P],
    "neuvv_shade": [ctypes.POINTER(neuvv_light), _P, _I64, _P, _P, _P, _P, _P, _P, _P],
    "neuvv_compose": [_I32, _I64, _P, _P, _P, _P, _P, _P, _P],
    "neuvv_compose_backward": [_I32, _I64, _P, _P, _P, _P, _P, _P, _P, _P],
    "neuvv_pinhole_rays": [ctypes.POINTER(neuvv_camera), _I64, _P, _P, _P, _P],
    "neuvv_eval_hh": [_I32, _I64, _P, _P, _P, _P],
}
EXPORTS = list(_SIGNATURES) + ["neuvv_last_error", "neuvv_version", "neuvv_trace_bytes", "neuvv_directory_entries"]

_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libneuvv.so (built by paper_2202_06088_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2202_06088_amd.build` "
                          "(the HIP library is required, there is no CPU fallback)")
    # torch ships its own HIP runtime; importing it first makes the library bind
    # to that copy (same soname) instead of loading a second runtime beside it,
    # which would see no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, args in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.neuvv_last_error.restype = ctypes.c_char_p
    lib.neuvv_last_error.argtypes = []
    lib.neuvv_version.restype = ctypes.c_int
    lib.neuvv_version.argtypes = []
    lib.neuvv_trace_bytes.restype = ctypes.c_int64
    lib.neuvv_trace_bytes.argtypes = [_I64, _I64]
    lib.neuvv_directory_entries.restype = ctypes.c_int64
    lib.neuvv_directory_entries.argtypes = [_I32]
    _lib = lib
    return lib


def _check(fn: str, rc: int):
    if rc != NEUVV_OK:
        msg = load().neuvv_last_error().decode(errors="replace")
        raise NeuvvError(fn, rc, msg)


def _ptr(t) -> Optional[int]:
    """data_ptr of a tensor (None stays NULL); ints pass through."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# one wrapper per exported call

def neuvv_version() -> int:
    return load().neuvv_version()


def neuvv_last_error() -> str:
    return load().neuvv_last_error().decode(errors="replace")


def neuvv_build_voctree(depth: int, leaf_ijk, nodes=None, node_capacity: int = 0, slot_of_input=None,
                        box_out=None) -> int:
    """leaf_ijk: host int32 numpy [N,3]; nodes: host int32 numpy [cap,4] or None;
    slot_of_input: host int64 numpy [N] or None; box_out: host int32 numpy [6] or None.
    Returns n_nodes."""
    n_nodes = ctypes.c_int64(0)
    n = 0 if leaf_ijk is None else int(leaf_ijk.shape[0])
    rc = load().neuvv_build_voctree(
        depth, n, None if leaf_ijk is None else leaf_ijk.ctypes.data,
        None if nodes is None else nodes.ctypes.data, int(node_capacity), ctypes.addressof(n_nodes),
        None if slot_of_input is None else slot_of_input.ctypes.data,
        None if box_out is None else box_out.ctypes.data)
    _check("neuvv_build_voctree", rc)
    return int(n_nodes.value)


def neuvv_payload_words(K: int, C: int, dtype: int, n_leaves: int):
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check("neuvv_payload_words",
           load().neuvv_payload_words(K, C, dtype, n_leaves, ctypes.addressof(a), ctypes.addressof(b)))
    return int(a.value), int(b.value)


def neuvv_pack_leaves(K, C, dtype, layout, n_leaves, hh_in, wsig_in, slot_of_input, hh_out, wsig_out,
                      stream=None):
    _check("neuvv_pack_leaves", load().neuvv_pack_leaves(K, C, dtype, layout, n_leaves, _ptr(hh_in), _ptr(wsig_in),
                                                         _ptr(slot_of_input), _ptr(hh_out), _ptr(wsig_out),
                                                         _stream(stream)))


def neuvv_pack_rows(R, dtype, layout, n_leaves, rows_in, slot_of_input, out, stream=None):
    _check("neuvv_pack_rows", load().neuvv_pack_rows(int(R), int(dtype), int(layout), int(n_leaves), _ptr(rows_in),
                                                     _ptr(slot_of_input), _ptr(out), _stream(stream)))


def _inst_ptr(inst: Optional[neuvv_instance]):
    return None if inst is None else ctypes.byref(inst)


def neuvv_render(tree: neuvv_tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop,
                 rgb, alpha, depth, nsamp, stream=None):
    _check("neuvv_render", load().neuvv_render(
        ctypes.byref(tree), _inst_ptr(inst), int(n_rays), _ptr(ray_o), _ptr(ray_d), _ptr(ray_t), float(t_scalar),
        int(image_width), float(t_stop), _ptr(rgb), _ptr(alpha), _ptr(depth), _ptr(nsamp), _stream(stream)))


def neuvv_render_noalloc(tree: neuvv_tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop,
                         rgb, alpha, depth, nsamp, stream=None):
    _check("neuvv_render_noalloc", load().neuvv_render_noalloc(
        ctypes.byref(tree), _inst_ptr(inst), int(n_rays), _ptr(ray_o), _ptr(ray_d), _ptr(ray_t), float(t_scalar),
        int(image_width), float(t_stop), _ptr(rgb), _ptr(alpha), _ptr(depth), _ptr(nsamp), _stream(stream)))


def neuvv_render_backward(tree: neuvv_tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop,
                          rgb, alpha, nsamp, grad_rgb, grad_alpha, grad_leaf, grad_basis, grad_basis_g=None,
                          stream=None):
    _check("neuvv_render_backward", load().neuvv_render_backward(
        ctypes.byref(tree), _inst_ptr(inst), int(n_rays), _ptr(ray_o), _ptr(ray_d), _ptr(ray_t), float(t_scalar),
        int(image_width), float(t_stop), _ptr(rgb), _ptr(alpha), _ptr(nsamp), _ptr(grad_rgb), _ptr(grad_alpha),
        _ptr(grad_leaf), _ptr(grad_basis), _ptr(grad_basis_g), _stream(stream)))


def neuvv_directory_entries(depth: int) -> int:
    v = load().neuvv_directory_entries(int(depth))
    if v < 0:
        raise NeuvvError("neuvv_directory_entries", -2, f"depth {depth} outside [1, 12]")
    return v


def neuvv_build_directory(depth, n_nodes, nodes, dir_out, capacity, stream=None):
    _check("neuvv_build_directory", load().neuvv_build_directory(int(depth), int(n_nodes), _ptr(nodes), _ptr(dir_out),
                                                                 int(capacity), _stream(stream)))


def neuvv_trace_bytes(n_rays: int, trace_cap: int) -> int:
    v = load().neuvv_trace_bytes(int(n_rays), int(trace_cap))
    if v < 0:
        raise NeuvvError("neuvv_trace_bytes", -1, "negative argument")
    return v


def neuvv_render_trace(tree: neuvv_tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop,
                       rgb, alpha, depth, nsamp, trace, trace_cap, stream=None):
    _check("neuvv_render_trace", load().neuvv_render_trace(
        ctypes.byref(tree), _inst_ptr(inst), int(n_rays), _ptr(ray_o), _ptr(ray_d), _ptr(ray_t), float(t_scalar),
        int(image_width), float(t_stop), _ptr(rgb), _ptr(alpha), _ptr(depth), _ptr(nsamp), _ptr(trace),
        int(trace_cap), _stream(stream)))


def neuvv_render_backward_trace(tree: neuvv_tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop,
                                rgb, alpha, nsamp, grad_rgb, grad_alpha, grad_leaf, grad_basis, grad_basis_g, trace,
                                trace_cap, stream=None):
    _check("neuvv_render_backward_trace", load().neuvv_render_backward_trace(
        ctypes.byref(tree), _inst_ptr(inst), int(n_rays), _ptr(ray_o), _ptr(ray_d), _ptr(ray_t), float(t_scalar),
        int(image_width), float(t_stop), _ptr(rgb), _ptr(alpha), _ptr(nsamp), _ptr(grad_rgb), _ptr(grad_alpha),
        _ptr(grad_leaf), _ptr(grad_basis), _ptr(grad_basis_g), _ptr(trace), int(trace_cap), _stream(stream)))


def neuvv_grad_row_elems(K: int, C: int, Cg: int = 0) -> int:
    rc = load().neuvv_grad_row_elems(int(K), int(C), int(Cg))
    if rc < 0:
        _check("neuvv_grad_row_elems", rc)
    return rc


def neuvv_compose(L, n_pix, rgb, alpha, depth, out_rgb, out_alpha, out_depth, stream=None):
    _check("neuvv_compose", load().neuvv_compose(int(L), int(n_pix), _ptr(rgb), _ptr(alpha), _ptr(depth),
                                                 _ptr(out_rgb), _ptr(out_alpha), _ptr(out_depth), _stream(stream)))


def neuvv_compose_backward(L, n_pix, rgb, alpha, depth, grad_out_rgb, grad_out_alpha, grad_rgb, grad_alpha,
                           stream=None):
    _check("neuvv_compose_backward", load().neuvv_compose_backward(
        int(L), int(n_pix), _ptr(rgb), _ptr(alpha), _ptr(depth), _ptr(grad_out_rgb), _ptr(grad_out_alpha),
        _ptr(grad_rgb), _ptr(grad_alpha), _stream(stream)))


def neuvv_pinhole_rays(cam: neuvv_camera, n, pix, ray_o, ray_d, stream=None):
    _check("neuvv_pinhole_rays", load().neuvv_pinhole_rays(ctypes.byref(cam), int(n), _ptr(pix), _ptr(ray_o),
                                                           _ptr(ray_d), _stream(stream)))


def neuvv_eval_hh(K, n, dirs, gam, out, stream=None):
    _check("neuvv_eval_hh", load().neuvv_eval_hh(int(K), int(n), _ptr(dirs), _ptr(gam), _ptr(out),
                                                 _stream(stream)))


def make_instance(rot, trans, scale=1.0, time_offset=0.0, wrap=False) -> neuvv_instance:
    inst = neuvv_instance()
    r = [float(x) for x in list(__import__("numpy").asarray(rot, dtype="float32").reshape(-1))]
    for i in range(9):
        inst.rot[i] = r[i]
    for i in range(3):
        inst.trans[i] = float(trans[i])
    inst.scale = float(scale)
    inst.time_offset = float(time_offset)
    inst.time_wrap = 1 if wrap else 0
    return inst


def make_camera(width, height, fx, fy, cx, cy, c2w) -> neuvv_camera:
    cam = neuvv_camera()
    cam.width, cam.height = int(width), int(height)
    cam.fx, cam.fy, cam.cx, cam.cy = float(fx), float(fy), float(cx), float(cy)
    flat = [float(x) for x in list(__import__("numpy").asarray(c2w, dtype="float32").reshape(-1))]
    for i in range(12):
        cam.c2w[i] = flat[i]
    return cam


def make_light(camera: neuvv_camera, ground_z, ground_rgb, background_rgb, shadow_strength, falloff_r0) -> neuvv_light:
    L = neuvv_light()
    L.camera = camera
    L.ground_z = float(ground_z)
    for i in range(3):
        L.ground_rgb[i] = float(ground_rgb[i])
        L.background_rgb[i] = float(background_rgb[i])
    L.shadow_strength = float(shadow_strength)
    L.falloff_r0 = float(falloff_r0)
    return L


def neuvv_blur(height, width, img_in, sigma, img_out, stream=None):
    _check("neuvv_blur", load().neuvv_blur(int(height), int(width), _ptr(img_in), float(sigma), _ptr(img_out),
                                           _stream(stream)))


def neuvv_shade(light: neuvv_light, shadow_map, n, ray_o, ray_d, rgb, alpha, depth, out_rgb, stream=None):
    _check("neuvv_shade", load().neuvv_shade(ctypes.byref(light), _ptr(shadow_map), int(n), _ptr(ray_o), _ptr(ray_d),
                                             _ptr(rgb), _ptr(alpha), _ptr(depth), _ptr(out_rgb), _stream(stream)))


def neuvv_find_terminal_leaves(tree: neuvv_tree, inst, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width,
                               alpha_threshold, last_leaf, stream=None):
    _check("neuvv_find_terminal_leaves", load().neuvv_find_terminal_leaves(
        ctypes.byref(tree), _inst_ptr(inst), int(n_rays), _ptr(ray_o), _ptr(ray_d), _ptr(ray_t), float(t_scalar),
        int(image_width), float(alpha_threshold), _ptr(last_leaf), _stream(stream)))


def neuvv_paint(n_rays, last_leaf, colours, sigma_d, t_d, n_leaves, edit, stream=None):
    _check("neuvv_paint", load().neuvv_paint(int(n_rays), _ptr(last_leaf), _ptr(colours), float(sigma_d), float(t_d),
                                             int(n_leaves), _ptr(edit), _stream(stream)))


def neuvv_render_multi(trees, insts, n_rays, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb, alpha, depth,
                       nsamp, stream=None):
    """trees: list of neuvv_tree structs; insts: list of neuvv_instance (or None = identity)."""
    L = len(trees)
    tarr = (ctypes.POINTER(neuvv_tree) * L)(*[ctypes.pointer(t) for t in trees])
    iarr = None
    if insts is not None:
        iarr = (neuvv_instance * L)(*[make_instance(np.eye(3), np.zeros(3), 1.0, 0.0, 0) if i is None else i
                                      for i in insts])
    _check("neuvv_render_multi", load().neuvv_render_multi(
        L, ctypes.cast(tarr, ctypes.c_void_p), None if iarr is None else ctypes.cast(iarr, ctypes.c_void_p),
        int(n_rays), _ptr(ray_o), _ptr(ray_d), _ptr(ray_t), float(t_scalar), int(image_width), float(t_stop),
        _ptr(rgb), _ptr(alpha), _ptr(depth), _ptr(nsamp), _stream(stream)))
