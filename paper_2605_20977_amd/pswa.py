"""Thin Python binding of libpswa.so (the C ABI in include/pswa.h).

Argument marshalling only: every step of the context model runs in the HIP
library. PyTorch provides device memory (tensors) and the current stream.
The functions keep the C names; each raises PswaError on a non-OK status.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: the library must bind to the HIP runtime torch already loaded
# (same soname), so that tensors, streams and kernels share one runtime.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpswa.so")

PSWA_FP32, PSWA_BF16, PSWA_FP8_E4M3 = 0, 1, 2
PSWA_SRC_DEVICE, PSWA_SRC_BITSTREAM = 0, 1
STATUS = {0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_ORDER", -4: "E_HIP",
          -5: "E_UNSUPPORTED", -6: "E_CORRUPT", -7: "E_NUMERIC"}
PRECISIONS = {"fp32": PSWA_FP32, "bf16": PSWA_BF16, "fp8": PSWA_FP8_E4M3}
PSWA_ACT_TENSOR, PSWA_ACT_ROW = 0, 1
ACT_SCALING = {"tensor": PSWA_ACT_TENSOR, "row": PSWA_ACT_ROW}


class PswaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pswa {STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class ModelDesc(C.Structure):
    _fields_ = [(n, C.c_int32) for n in
                ("L", "d", "heads", "window", "mlp_ratio", "C", "Ch", "prec", "cycle",
                 "act_scaling", "ch_groups", "ch_d", "ch_L", "ch_ratio")]


class FrameDesc(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("H", "W", "Hh", "Wh", "n_prev")]


class BatchFrame(C.Structure):
    _fields_ = [("frame", FrameDesc), ("d_hyper", C.c_void_p), ("d_prev", C.c_void_p),
                ("d_latents", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built: run `python -m paper_2605_20977_amd.build` "
            "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, sz, i32 = C.c_void_p, C.c_size_t, C.c_int
    P = C.POINTER
    sig = {
        "pswa_model_blob_floats": (sz, [P(ModelDesc)]),
        "pswa_act_points": (i32, [P(ModelDesc)]),
        "pswa_calibrate_workspace_bytes": (sz, [vp, P(FrameDesc)]),
        "pswa_calibrate": (i32, [vp, P(FrameDesc), vp, vp, vp, vp, vp, sz, vp]),
        "pswa_noalloc_scratch_bytes": (sz, []),
        "pswa_encode_params_noalloc": (i32, [vp, P(FrameDesc), vp, vp, vp, vp, vp, vp, vp, vp,
                                             P(C.c_double), vp]),
        "pswa_model_device_bytes": (sz, [P(ModelDesc)]),
        "pswa_model_create": (i32, [P(ModelDesc), vp, sz, vp, sz, vp, P(vp)]),
        "pswa_model_destroy": (None, [vp]),
        "pswa_encode_workspace_bytes": (sz, [vp, P(FrameDesc)]),
        "pswa_encode_params": (i32, [vp, P(FrameDesc), vp, vp, vp, vp, vp, vp, vp, vp,
                                     P(C.c_double), vp, sz, vp]),
        "pswa_state_bytes": (sz, [vp, P(FrameDesc)]),
        "pswa_decode_begin": (i32, [vp, P(FrameDesc), vp, vp, i32, vp, sz, vp, sz, vp, P(vp)]),
        "pswa_num_steps": (i32, [vp]),
        "pswa_decode_step": (i32, [vp, i32, vp]),
        "pswa_decode_end": (i32, [vp, vp, vp, vp, vp, vp, vp, P(C.c_double), vp]),
        "pswa_state_destroy": (None, [vp]),
        "pswa_cdf_select": (i32, [vp, vp, sz, vp, vp, vp]),
        "pswa_cdf_tables": (i32, [vp, vp, vp, sz]),
        "pswa_range_encode": (i32, [P(FrameDesc), C.c_int32, C.c_int32, C.c_int32, vp, vp, vp,
                                    vp, sz, P(sz)]),
        "pswa_range_encode_seq": (i32, [sz, vp, vp, vp, vp, sz, P(sz)]),
        "pswa_range_decode_seq": (i32, [vp, sz, sz, vp, vp, vp]),
        "pswa_last_error": (C.c_char_p, []),
        "pswa_batch_workspace_bytes": (sz, [vp, i32, P(BatchFrame)]),
        "pswa_batch_create": (i32, [vp, i32, P(BatchFrame), i32, vp, sz, vp, P(vp)]),
        "pswa_batch_run": (i32, [vp, vp]),
        "pswa_batch_check": (i32, [vp, vp]),
        "pswa_batch_outputs": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, P(C.c_double), vp]),
        "pswa_batch_num_steps": (i32, [vp]),
        "pswa_batch_max_rows": (i32, [vp]),
        "pswa_batch_grid": (i32, [vp]),
        "pswa_batch_max_grid": (i32, [vp]),
        "pswa_batch_set_grid": (i32, [vp, i32]),
        "pswa_batch_set_spin_limit": (i32, [vp, C.c_int64]),
        "pswa_batch_trace": (i32, [vp, vp, i32]),
        "pswa_batch_set_rtile": (i32, [vp, i32]),
        "pswa_batch_rtile": (i32, [vp]),
        "pswa_batch_autotune": (i32, [vp, C.c_char_p, i32, vp, P(i32), P(i32), P(i32),
                                      P(C.c_float)]),
        "pswa_batch_set_groups": (i32, [vp, i32, i32, vp]),
        "pswa_batch_set_xcd_barrier": (i32, [vp, i32]),
        "pswa_batch_set_attention": (i32, [vp, i32]),
        "pswa_batch_attention": (i32, [vp]),
        "pswa_train_workspace_bytes": (sz, [P(ModelDesc), i32, i32, i32]),
        "pswa_train_create": (i32, [P(ModelDesc), vp, sz, i32, i32, i32, vp, sz, vp, P(vp)]),
        "pswa_train_step": (i32, [vp, i32, i32, vp, vp, vp, vp, vp, C.c_float, C.c_float, i32,
                                  P(C.c_double), vp]),
        "pswa_train_read": (i32, [vp, i32, vp, sz, vp]),
        "pswa_train_num_steps": (i32, [vp]),
        "pswa_train_destroy": (None, [vp]),
        "pswa_student_accept": (i32, [C.c_double, C.c_double, C.c_double]),
        "pswa_batch_groups": (i32, [vp, P(i32), P(i32), P(i32)]),
        "pswa_batch_capture": (i32, [vp, vp]),
        "pswa_batch_destroy": (None, [vp]),
        "pswa_quantize": (i32, [i32, vp, sz, vp, P(C.c_float)]),
        "pswa_profile_enable": (i32, [i32]),
        "pswa_profile_roles": (i32, []),
        "pswa_profile_read": (i32, [i32, C.c_char_p, sz, P(C.c_double), P(C.c_int64),
                                    P(C.c_double), P(C.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("pswa_model_blob_floats", "pswa_model_device_bytes", "pswa_model_create",
            "pswa_model_destroy", "pswa_encode_workspace_bytes", "pswa_encode_params",
            "pswa_state_bytes", "pswa_decode_begin", "pswa_num_steps", "pswa_decode_step",
            "pswa_decode_end", "pswa_state_destroy", "pswa_cdf_select", "pswa_cdf_tables",
            "pswa_range_encode", "pswa_range_encode_seq", "pswa_range_decode_seq",
            "pswa_last_error", "pswa_profile_enable", "pswa_profile_roles", "pswa_profile_read",
            "pswa_batch_workspace_bytes", "pswa_batch_create", "pswa_batch_run",
            "pswa_batch_check", "pswa_batch_outputs", "pswa_batch_num_steps",
            "pswa_batch_max_rows", "pswa_batch_grid", "pswa_batch_max_grid",
            "pswa_batch_set_grid", "pswa_batch_set_spin_limit", "pswa_batch_destroy",
            "pswa_quantize", "pswa_batch_trace", "pswa_batch_set_rtile", "pswa_batch_rtile",
            "pswa_batch_autotune", "pswa_batch_capture", "pswa_batch_set_groups",
            "pswa_batch_groups", "pswa_train_workspace_bytes", "pswa_train_create",
            "pswa_train_step", "pswa_train_read", "pswa_train_num_steps", "pswa_train_destroy",
            "pswa_student_accept", "pswa_batch_set_xcd_barrier", "pswa_act_points",
            "pswa_calibrate_workspace_bytes", "pswa_calibrate", "pswa_noalloc_scratch_bytes",
            "pswa_encode_params_noalloc", "pswa_batch_set_attention", "pswa_batch_attention")


def lib():
    return _lib


def _check(st):
    if st != 0:
        raise PswaError(st, _lib.pswa_last_error().decode())


def _ptr(t):
    """Device/host address of a tensor or numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ shapes

def model_desc(cfg, prec="fp32", act="tensor") -> ModelDesc:
    cg = getattr(cfg, "ch_groups", 0)
    return ModelDesc(cfg.L, cfg.d, cfg.heads, cfg.window, cfg.mlp_ratio, cfg.C, cfg.Ch,
                     PRECISIONS[prec] if isinstance(prec, str) else int(prec),
                     getattr(cfg, "cycle", 0), ACT_SCALING[act], cg,
                     cfg.ch_d if cg else 0, cfg.ch_L if cg else 0, cfg.ch_ratio if cg else 0)


def frame_desc(H, W, n_prev=0) -> FrameDesc:
    return FrameDesc(H, W, -(-H // 4), -(-W // 4), n_prev)


def blob_shapes(cfg) -> list[tuple[str, tuple]]:
    """(name, shape) of every parameter in the blob order the header
    documents; linear weights are [out_features][in_features]."""
    d, C, Ch, F, h, r = cfg.d, cfg.C, cfg.Ch, cfg.mlp_ratio * cfg.d, cfg.heads, (cfg.window - 1) // 2
    k2 = (2 * r + 1) ** 2
    if getattr(cfg, "cycle", 0):   # full window for the cyclic schedule
        n_acc, n_lay = k2, k2 + 2 * k2
    else:
        n_acc = 2 * r * (r + 1)
        n_lay = n_acc + 1 + 2 * k2
    out = [("hyper.W", (d, Ch)), ("hyper.P4", (16, d)), ("in.g", (C,)), ("in.W", (d, C)),
           ("acc.gq", (d,)), ("acc.Wq", (d, d)), ("acc.gkv", (d,)), ("acc.Wkv", (2 * d, d)),
           ("acc.knull", (d,)), ("acc.vnull", (d,)), ("acc.bias", (h, n_acc)),
           ("acc.Wo", (d, d))]
    for l in range(cfg.L):
        p = f"layer{l}."
        out += [(p + "g1", (d,)), (p + "Wqkv", (3 * d, d)), (p + "bias", (h, n_lay)),
                (p + "Wo", (d, d)), (p + "g2", (d,)), (p + "Wgate", (F, d)),
                (p + "Wup", (F, d)), (p + "Wdown", (d, F))]
    N = getattr(cfg, "ch_groups", 0)
    if N:  # Channel Transformer and grouped heads in place of the plain head
        dc = cfg.ch_d
        dg, Cg = dc // N, C // N
        Fg = cfg.ch_ratio * dg
        out += [("ct.gx", (d,)), ("ct.Wx", (dc, d)), ("ct.gy", (C,)), ("ct.Wy", (dc, C))]
        for b in range(cfg.ch_L):
            p = f"ct{b}."
            out += [(p + "g1", (dc,)), (p + "M", (dc, dc)), (p + "g2", (dc,)),
                    (p + "Wgate", (N, Fg, dg)), (p + "Wup", (N, Fg, dg)),
                    (p + "Wdown", (N, dg, Fg))]
        out += [("ctH.g", (dc,)), ("ctH.W1", (N, dg, dg)), ("ctH.W2", (N, 2 * Cg, dg))]
    else:
        out += [("head.g", (d,)), ("head.W1", (d, d)), ("head.W2", (2 * C, d))]
    out += [("head.gmu", (C,)), ("head.bmu", (C,)), ("head.gsig", (C,)), ("head.bsig", (C,))]
    return out


def blob_order(cfg) -> list[str]:
    """Parameter names in the blob order the header documents."""
    return [n for n, _ in blob_shapes(cfg)]


def pack_blob(cfg, weights) -> np.ndarray:
    return np.concatenate([np.asarray(weights[n], dtype=np.float32).ravel()
                           for n in blob_order(cfg)])


def unpack_blob(cfg, blob) -> dict:
    """Inverse of pack_blob: {name: float32 array of its shape}."""
    out, off = {}, 0
    for name, shape in blob_shapes(cfg):
        n = int(np.prod(shape))
        out[name] = np.asarray(blob[off:off + n], dtype=np.float32).reshape(shape).copy()
        off += n
    return out


# ------------------------------------------------------------------- model

class Model:
    """A model uploaded into a torch-owned device region.

    FP8 models scale their projection inputs per tensor (act='tensor', the
    default), from the calibrated maxima act_amax (see calibrate), or per row
    (act='row')."""

    def __init__(self, cfg, weights, prec="fp32", device="cuda", act="tensor", act_amax=None):
        import torch
        self.cfg = cfg
        fp8 = (PRECISIONS[prec] if isinstance(prec, str) else int(prec)) == PSWA_FP8_E4M3
        self.act = act if fp8 else "tensor"
        self.desc = model_desc(cfg, prec, self.act)
        blob = pack_blob(cfg, weights)
        if fp8 and self.act == "tensor":
            if act_amax is None:
                raise PswaError(-1, "an FP8 per-tensor model needs calibrated act_amax")
            blob = np.concatenate([blob, np.asarray(act_amax, dtype=np.float32).ravel()])
        self.act_amax = None if act_amax is None else np.asarray(act_amax, np.float32)
        need = _lib.pswa_model_blob_floats(C.byref(self.desc))
        if need != blob.size:
            raise PswaError(-2, f"blob has {blob.size} floats, library expects {need}")
        nbytes = _lib.pswa_model_device_bytes(C.byref(self.desc))
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(_lib.pswa_model_create(C.byref(self.desc), blob.ctypes.data, blob.size,
                                      _ptr(self.mem), nbytes, _stream(), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pswa_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def _i32(t, device):
    import torch
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t, dtype=np.int32))
    return t.to(device=device, dtype=torch.int32).contiguous()


def _shape_check(model, y=None, z=None, prev=None, H=None, W=None):
    """Refuse mis-shaped tensors before any pointer reaches the library."""
    cfg = model.cfg
    if y is not None:
        if y.dim() != 3 or y.shape[2] != cfg.C:
            raise PswaError(-2, f"latents must be [H][W][{cfg.C}], got {tuple(y.shape)}")
        H, W = y.shape[0], y.shape[1]
    if z is not None and tuple(z.shape) != (-(-H // 4), -(-W // 4), cfg.Ch):
        raise PswaError(-2, f"hyperprior must be [{-(-H // 4)}][{-(-W // 4)}][{cfg.Ch}], "
                            f"got {tuple(z.shape)}")
    if prev is not None and tuple(prev.shape) != (2, H, W, cfg.C):
        raise PswaError(-2, f"previous latents must be [2][{H}][{W}][{cfg.C}], "
                            f"got {tuple(prev.shape)}")


def _outputs(H, W, Cc, device):
    import torch
    n = (H, W, Cc)
    return {
        "mean": torch.empty(n, dtype=torch.float32, device=device),
        "scale": torch.empty(n, dtype=torch.float32, device=device),
        "bits": torch.empty(n, dtype=torch.float32, device=device),
        "center": torch.empty(n, dtype=torch.int32, device=device),
        "index": torch.empty(n, dtype=torch.int16, device=device),  # holds uint16 bits
    }


def pswa_encode_params(model: Model, latents, hyper, prev=None, total_bits=True, ws=None):
    """Parallel encode form. Returns dict of device tensors (index holds the
    uint16 table index in an int16 tensor; use index_u16()) and 'total_bits'."""
    import torch
    dev = model.mem.device
    y = _i32(latents, dev)
    z = _i32(hyper, dev)
    H, W, Cc = y.shape
    pv = _i32(prev, dev) if prev is not None else None
    _shape_check(model, y, z, pv)
    fd = frame_desc(H, W, 2 if pv is not None else 0)
    nws = _lib.pswa_encode_workspace_bytes(model.handle, C.byref(fd))
    if nws == 0:
        raise PswaError(-2, "invalid frame for this model")
    if ws is None or ws.numel() < nws:
        ws = torch.empty(nws, dtype=torch.uint8, device=dev)
    out = _outputs(H, W, Cc, dev)
    tot = C.c_double(0.0)
    _check(_lib.pswa_encode_params(
        model.handle, C.byref(fd), _ptr(y), _ptr(z), _ptr(pv), _ptr(out["mean"]),
        _ptr(out["scale"]), _ptr(out["bits"]), _ptr(out["center"]), _ptr(out["index"]),
        C.byref(tot) if total_bits else None, _ptr(ws), ws.numel(), _stream()))
    if total_bits:
        out["total_bits"] = tot.value
    return out


def pswa_encode_params_noalloc(model: Model, latents, hyper, prev=None, total_bits=True,
                               out=None):
    """The encode form on the library's static scratch (no workspace is
    allocated by the library or here); out: optional preallocated outputs
    (dict as returned)."""
    dev = model.mem.device
    y = _i32(latents, dev)
    z = _i32(hyper, dev)
    H, W, Cc = y.shape
    pv = _i32(prev, dev) if prev is not None else None
    _shape_check(model, y, z, pv)
    fd = frame_desc(H, W, 2 if pv is not None else 0)
    out = out or _outputs(H, W, Cc, dev)
    tot = C.c_double(0.0)
    _check(_lib.pswa_encode_params_noalloc(
        model.handle, C.byref(fd), _ptr(y), _ptr(z), _ptr(pv), _ptr(out["mean"]),
        _ptr(out["scale"]), _ptr(out["bits"]), _ptr(out["center"]), _ptr(out["index"]),
        C.byref(tot) if total_bits else None, _stream()))
    if total_bits:
        out["total_bits"] = tot.value
    return out


class State:
    def __init__(self, handle, mem, keep):
        self.handle = handle
        self.mem = mem
        self._keep = keep
        self.T = _lib.pswa_num_steps(handle)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pswa_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def pswa_state_bytes(model: Model, H, W, n_prev=0):
    fd = frame_desc(H, W, n_prev)
    return _lib.pswa_state_bytes(model.handle, C.byref(fd))


def pswa_decode_begin(model: Model, H, W, hyper, prev=None, source="device", src=None,
                      mem=None):
    """src: device latents (source='device') or bytes (source='bitstream')."""
    import torch
    dev = model.mem.device
    z = _i32(hyper, dev)
    pv = _i32(prev, dev) if prev is not None else None
    _shape_check(model, None, z, pv, H, W)
    fd = frame_desc(H, W, 2 if pv is not None else 0)
    nb = _lib.pswa_state_bytes(model.handle, C.byref(fd))
    if nb == 0:
        raise PswaError(-2, "invalid frame for this model")
    if mem is None or mem.numel() < nb:
        mem = torch.empty(nb, dtype=torch.uint8, device=dev)
    keep = [z, pv]
    if source == "device":
        s = _i32(src, dev)
        if tuple(s.shape) != (H, W, model.cfg.C):
            raise PswaError(-2, f"device symbol source must be [{H}][{W}][{model.cfg.C}]")
        keep.append(s)
        kind, sp, sn = PSWA_SRC_DEVICE, _ptr(s), s.numel() * 4
    elif source == "bitstream":
        buf = np.frombuffer(bytes(src), dtype=np.uint8).copy()
        keep.append(buf)
        kind, sp, sn = PSWA_SRC_BITSTREAM, buf.ctypes.data, buf.size
    else:
        raise ValueError(source)
    h = C.c_void_p()
    _check(_lib.pswa_decode_begin(model.handle, C.byref(fd), _ptr(z), _ptr(pv), kind, sp, sn,
                                  _ptr(mem), mem.numel(), _stream(), C.byref(h)))
    return State(h, mem, keep)


def pswa_num_steps(state: State) -> int:
    return _lib.pswa_num_steps(state.handle)


def pswa_decode_step(state: State, t: int):
    _check(_lib.pswa_decode_step(state.handle, t, _stream()))


def pswa_decode_end(state: State, H, W, Cc, total_bits=True):
    import torch
    dev = state.mem.device
    out = _outputs(H, W, Cc, dev)
    out["latents"] = torch.empty((H, W, Cc), dtype=torch.int32, device=dev)
    tot = C.c_double(0.0)
    _check(_lib.pswa_decode_end(state.handle, _ptr(out["latents"]), _ptr(out["mean"]),
                                _ptr(out["scale"]), _ptr(out["bits"]), _ptr(out["center"]),
                                _ptr(out["index"]), C.byref(tot) if total_bits else None,
                                _stream()))
    if total_bits:
        out["total_bits"] = tot.value
    return out


def decode_frame(model: Model, H, W, hyper, prev=None, source="device", src=None, mem=None):
    st = pswa_decode_begin(model, H, W, hyper, prev, source, src, mem)
    for t in range(st.T):
        pswa_decode_step(st, t)
    out = pswa_decode_end(st, H, W, model.cfg.C)
    st.close()
    return out


def index_u16(t):
    """uint16 numpy view of an index tensor."""
    return t.cpu().numpy().view(np.uint16)


# ---------------------------------------------------------- batched decode

class Batch:
    """Persistent decode of many frames in one launch.

    frames: list of dict(latents=[H][W][C], hyper=[Hh][Wh][Ch], prev=None or
    [2][H][W][C]) as numpy arrays or tensors (moved to the model's device)."""

    def __init__(self, model: Model, frames, grid=0):
        import torch
        self.model = model
        dev = model.mem.device
        self._keep = []
        arr = (BatchFrame * len(frames))()
        self.shapes = []
        for k, f in enumerate(frames):
            y = _i32(f["latents"], dev)
            z = _i32(f["hyper"], dev)
            pv = _i32(f["prev"], dev) if f.get("prev") is not None else None
            _shape_check(model, y, z, pv)
            H, W = y.shape[0], y.shape[1]
            self.shapes.append((H, W))
            self._keep += [y, z, pv]
            arr[k].frame = frame_desc(H, W, 2 if pv is not None else 0)
            arr[k].d_hyper = _ptr(z)
            arr[k].d_prev = _ptr(pv)
            arr[k].d_latents = _ptr(y)
        self._frames = arr
        nb = _lib.pswa_batch_workspace_bytes(model.handle, len(frames), arr)
        if nb == 0:
            raise PswaError(-2, "invalid batch: " + _lib.pswa_last_error().decode())
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        _check(_lib.pswa_batch_create(model.handle, len(frames), arr, grid, _ptr(self.ws), nb,
                                      _stream(), C.byref(h)))
        self.handle = h
        self.T = _lib.pswa_batch_num_steps(h)
        self.max_rows = _lib.pswa_batch_max_rows(h)

    @property
    def grid(self):
        return _lib.pswa_batch_grid(self.handle)

    @property
    def max_grid(self):
        return _lib.pswa_batch_max_grid(self.handle)

    def set_grid(self, g):
        _check(_lib.pswa_batch_set_grid(self.handle, int(g)))

    def inputs(self, k):
        """Device tensors (latents, hyper, prev or None) that frame k reads."""
        return tuple(self._keep[3 * k:3 * k + 3])

    @property
    def rtile(self):
        return _lib.pswa_batch_rtile(self.handle)

    def set_rtile(self, r):
        _check(_lib.pswa_batch_set_rtile(self.handle, int(r)))

    def autotune(self, cache_path=None, reps=3):
        """Pick the grouping and row tile by timing; returns (frames per
        group, blocks per group, rtile, estimated ms per run)."""
        f, g, r, ms = C.c_int(), C.c_int(), C.c_int(), C.c_float()
        _check(_lib.pswa_batch_autotune(self.handle,
                                        cache_path.encode() if cache_path else None, reps,
                                        _stream(), C.byref(f), C.byref(g), C.byref(r),
                                        C.byref(ms)))
        return f.value, g.value, r.value, ms.value

    def set_attention(self, staged):
        """Attention form: True = LDS-staged window tiles, False = keys from
        global memory (same bits)."""
        _check(_lib.pswa_batch_set_attention(self.handle, 1 if staged else 0))

    @property
    def attention_staged(self):
        return _lib.pswa_batch_attention(self.handle) == 1

    def set_xcd_barrier(self, on):
        _check(_lib.pswa_batch_set_xcd_barrier(self.handle, 1 if on else 0))

    def set_groups(self, frames_per_group, blocks_per_group):
        _check(_lib.pswa_batch_set_groups(self.handle, int(frames_per_group),
                                          int(blocks_per_group), _stream()))

    @property
    def groups(self):
        """(frames per group, blocks per group, number of groups)."""
        f, g, n = C.c_int(), C.c_int(), C.c_int()
        _check(_lib.pswa_batch_groups(self.handle, C.byref(f), C.byref(g), C.byref(n)))
        return f.value, g.value, n.value

    def capture(self):
        """Record one run into a HIP graph; later run() calls replay it."""
        _check(_lib.pswa_batch_capture(self.handle, _stream()))

    def set_spin_limit(self, n):
        _check(_lib.pswa_batch_set_spin_limit(self.handle, int(n)))

    def set_trace(self, buf):
        """buf: int64 device tensor (or None to stop tracing)."""
        _check(_lib.pswa_batch_trace(self.handle, _ptr(buf), 0 if buf is None else buf.numel()))

    def run(self):
        _check(_lib.pswa_batch_run(self.handle, _stream()))

    def check(self):
        _check(_lib.pswa_batch_check(self.handle, _stream()))

    def outputs(self, f, total_bits=True):
        import torch
        H, W = self.shapes[f]
        dev = self.ws.device
        out = _outputs(H, W, self.model.cfg.C, dev)
        out["latents"] = torch.empty((H, W, self.model.cfg.C), dtype=torch.int32, device=dev)
        tot = C.c_double(0.0)
        _check(_lib.pswa_batch_outputs(self.handle, f, _ptr(out["latents"]), _ptr(out["mean"]),
                                       _ptr(out["scale"]), _ptr(out["bits"]),
                                       _ptr(out["center"]), _ptr(out["index"]),
                                       C.byref(tot) if total_bits else None, _stream()))
        if total_bits:
            out["total_bits"] = tot.value
        return out

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pswa_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


# ------------------------------------------------------------ entropy side

def pswa_cdf_select(mean, log_scale):
    import torch
    n = mean.numel()
    c = torch.empty(n, dtype=torch.int32, device=mean.device)
    i = torch.empty(n, dtype=torch.int16, device=mean.device)
    _check(_lib.pswa_cdf_select(_ptr(mean), _ptr(log_scale), n, _ptr(c), _ptr(i), _stream()))
    return c, i


def pswa_cdf_tables():
    """(radius uint32 [1024], offset uint32 [1025], freq uint16 [..]) on the host."""
    off = np.zeros(1025, np.uint32)
    rad = np.zeros(1024, np.uint32)
    _check(_lib.pswa_cdf_tables(rad.ctypes.data, off.ctypes.data, None, 0))
    freq = np.zeros(int(off[1024]), np.uint16)
    _check(_lib.pswa_cdf_tables(rad.ctypes.data, off.ctypes.data, freq.ctypes.data, freq.size))
    return rad, off, freq


def _u8cap(n_symbols):
    return 64 + 8 * n_symbols


def pswa_range_encode(H, W, Cc, window, symbols, center, index, cycle=0) -> bytes:
    """Range-code [H][W][C] symbols in the decode order of the schedule
    (window and cycle of the model)."""
    fd = frame_desc(H, W, 0)
    sy = np.ascontiguousarray(symbols, dtype=np.int32)
    ce = np.ascontiguousarray(center, dtype=np.int32)
    ix = np.ascontiguousarray(index).view(np.uint16)
    cap = _u8cap(sy.size)
    out = np.empty(cap, np.uint8)
    nb = C.c_size_t(0)
    _check(_lib.pswa_range_encode(C.byref(fd), Cc, window, int(cycle), sy.ctypes.data,
                                  ce.ctypes.data, ix.ctypes.data, out.ctypes.data, cap,
                                  C.byref(nb)))
    return out[:nb.value].tobytes()


def pswa_range_encode_seq(symbols, center, index) -> bytes:
    sy = np.ascontiguousarray(symbols, dtype=np.int32).ravel()
    ce = np.ascontiguousarray(center, dtype=np.int32).ravel()
    ix = np.ascontiguousarray(index).view(np.uint16).ravel()
    cap = _u8cap(sy.size)
    out = np.empty(cap, np.uint8)
    nb = C.c_size_t(0)
    _check(_lib.pswa_range_encode_seq(sy.size, sy.ctypes.data, ce.ctypes.data, ix.ctypes.data,
                                      out.ctypes.data, cap, C.byref(nb)))
    return out[:nb.value].tobytes()


def pswa_range_decode_seq(data: bytes, center, index):
    ce = np.ascontiguousarray(center, dtype=np.int32).ravel()
    ix = np.ascontiguousarray(index).view(np.uint16).ravel()
    buf = np.frombuffer(data, dtype=np.uint8).copy()
    out = np.empty(ce.size, np.int32)
    _check(_lib.pswa_range_decode_seq(buf.ctypes.data if buf.size else None, buf.size,
                                      ce.size, ce.ctypes.data, ix.ctypes.data,
                                      out.ctypes.data))
    return out


# ------------------------------------------------------------ quantization

def pswa_quantize(prec, x):
    """(codes, inv_scale): uint16 BF16 bits or uint8 FP8 e4m3fn codes."""
    a = np.ascontiguousarray(x, dtype=np.float32).ravel()
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    out = np.empty(a.size, np.uint16 if p == PSWA_BF16 else np.uint8)
    inv = C.c_float(0)
    _check(_lib.pswa_quantize(p, a.ctypes.data, a.size, out.ctypes.data, C.byref(inv)))
    return out, inv.value


# --------------------------------------------------------------- profiling

def pswa_profile_enable(on: bool):
    _check(_lib.pswa_profile_enable(1 if on else 0))


def pswa_profile_read():
    """{role: dict(ms, launches, bytes, flops)} for roles with launches."""
    out = {}
    name = C.create_string_buffer(64)
    ms, n = C.c_double(), C.c_int64()
    by, fl = C.c_double(), C.c_double()
    for r in range(_lib.pswa_profile_roles()):
        _check(_lib.pswa_profile_read(r, name, 64, C.byref(ms), C.byref(n), C.byref(by),
                                      C.byref(fl)))
        if n.value:
            out[name.value.decode()] = {"ms": ms.value, "launches": n.value,
                                        "bytes": by.value, "flops": fl.value}
    return out


# ---------------------------------------------------------------- training

class Trainer:
    """Distillation trainer of a (student) model: FP32 weights, gradients
    and AdamW moments in a torch-owned device region; crops of H x W."""

    def __init__(self, cfg, weights, max_crops, H, W, device="cuda"):
        import torch
        self.cfg, self.H, self.W, self.max_crops = cfg, H, W, max_crops
        self.desc = model_desc(cfg, "fp32")
        blob = pack_blob(cfg, weights)
        nb = _lib.pswa_train_workspace_bytes(C.byref(self.desc), max_crops, H, W)
        if nb == 0:
            raise PswaError(-2, "invalid trainer shape")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(_lib.pswa_train_create(C.byref(self.desc), blob.ctypes.data, blob.size, max_crops,
                                      H, W, _ptr(self.ws), nb, _stream(), C.byref(h)))
        self.handle = h
        self.blob_floats = blob.size

    def step(self, latents, hyper, mu_t, lsig_t, prev=None, lr=1e-3, weight_decay=0.0,
             update=True):
        """One step on device tensors latents [B][H][W][C] (int32), hyper
        [B][Hh][Wh][Ch] (int32), prev [B][2][H][W][C] or None, targets
        [B][H][W][C] (float32). Returns the loss."""
        B = latents.shape[0]
        loss = C.c_double()
        _check(_lib.pswa_train_step(self.handle, B, 2 if prev is not None else 0,
                                    _ptr(latents), _ptr(hyper), _ptr(prev), _ptr(mu_t),
                                    _ptr(lsig_t), float(lr), float(weight_decay),
                                    1 if update else 0, C.byref(loss), _stream()))
        return loss.value

    def read(self, what="weights"):
        blob = np.empty(self.blob_floats, dtype=np.float32)
        _check(_lib.pswa_train_read(self.handle, 0 if what == "weights" else 1,
                                    blob.ctypes.data, blob.size, _stream()))
        return unpack_blob(self.cfg, blob)

    @property
    def steps(self):
        return _lib.pswa_train_num_steps(self.handle)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pswa_train_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def pswa_student_accept(bits_student, bits_full, max_overhead=0.01):
    """True when a frame keeps the student: its bits exceed the full model's
    by at most max_overhead (a fraction)."""
    return bool(_lib.pswa_student_accept(float(bits_student), float(bits_full),
                                         float(max_overhead)))


def pswa_act_points(cfg) -> int:
    return _lib.pswa_act_points(C.byref(model_desc(cfg)))


def pswa_calibrate(model: Model, frames):
    """Maxima of every projection input of the FP32 model over the frames
    (dicts with latents, hyper, prev): float32 numpy [pswa_act_points]."""
    import torch
    dev = model.mem.device
    amax = torch.zeros(pswa_act_points(model.cfg), dtype=torch.float32, device=dev)
    ws = None
    for f in frames:
        y = _i32(f["latents"], dev)
        z = _i32(f["hyper"], dev)
        pv = _i32(f["prev"], dev) if f.get("prev") is not None else None
        _shape_check(model, y, z, pv)
        fd = frame_desc(y.shape[0], y.shape[1], 2 if pv is not None else 0)
        nws = _lib.pswa_calibrate_workspace_bytes(model.handle, C.byref(fd))
        if ws is None or ws.numel() < nws:
            ws = torch.empty(nws, dtype=torch.uint8, device=dev)
        _check(_lib.pswa_calibrate(model.handle, C.byref(fd), _ptr(y), _ptr(z), _ptr(pv),
                                   _ptr(amax), _ptr(ws), ws.numel(), _stream()))
    torch.cuda.current_stream().synchronize()
    return amax.cpu().numpy()


def make_model(cfg, weights, prec="fp32", calib_frames=None, act="tensor", device="cuda"):
    """A model in the given arithmetic, ready to run. An FP8 per-tensor
    model is calibrated first, with the FP32 model, on calib_frames."""
    if prec == "fp8" and act == "tensor":
        if not calib_frames:
            raise PswaError(-1, "an FP8 per-tensor model needs calibration frames")
        ref = Model(cfg, weights, "fp32", device)
        amax = pswa_calibrate(ref, calib_frames)
        ref.close()
        return Model(cfg, weights, prec, device, act="tensor", act_amax=amax)
    return Model(cfg, weights, prec, device, act=act)
