"""Thin ctypes binding of libsiting.so (include/siting.h).

Argument marshalling only: each function has the C name, takes torch tensors
that already live on the HIP device, passes their data pointers and the
current torch stream, and raises SitingError on a non-zero return code.
Torch provides device memory and streams; every step of the siting path runs
in the library's HIP kernels.  There is no fallback: if libsiting.so is
missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsiting.so")

SITING_OK = 0
SITING_KEY_U8, SITING_KEY_F32 = 0, 1
SITING_SINK_BITMAP, SITING_SINK_COUNT = 0, 1

OBSERVER_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("roi", "<i4"),
                           ("h_t", "<i4"), ("h_r", "<i4")])


class SitingError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


class Schedule(C.Structure):
    _fields_ = [("waves", C.c_int32), ("groups_per_cu", C.c_int32),
                ("stage_rmax", C.c_int32), ("ray_per_wave", C.c_int32)]

    def as_tuple(self):
        return (self.waves, self.groups_per_cu, self.stage_rmax, self.ray_per_wave)

    def __repr__(self):
        return ("Schedule(waves=%d, groups_per_cu=%d, stage_rmax=%d, ray_per_wave=%d)"
                % self.as_tuple())


def _load():
    # torch ships its own HIP runtime under the same soname as the system
    # one; loading torch first makes libsiting bind to that single runtime
    # instead of bringing a second one into the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2006_16783_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P, i64, i32, u64, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_size_t
    sig = {
        "siting_abi_version": ([], C.c_int),
        "siting_last_error": ([], C.c_char_p),
        "siting_device_cus": ([P], C.c_int),
        "siting_vix": ([P, i64, i64, i64, i32, i32, i32, i32, u64, P, P], C.c_int),
        "siting_vix_stats": ([P, i64, i64, i64, i32, i32, i32, i32, u64, P, P, P], C.c_int),
        "siting_findmax": ([P, i32, i32, P, i64, i64, i64, i32, i32, i32, P, P], C.c_int),
        "siting_viewshed_layout": ([P, i64, i64, i64, P], i64),
        "siting_viewshed_order": ([P, i64, P], C.c_int),
        "siting_viewshed_workspace_size": ([], sz),
        "siting_viewshed_default_schedule": ([i32, P], C.c_int),
        "siting_viewshed_batch": ([P, i64, i64, i64, P, i64, P, P, i32, P, i32, P, P, P, P, sz, P],
                                  C.c_int),
        "siting_viewshed_r3": ([P, i64, i64, i64, P, i64, P, P, P], C.c_int),
        "siting_visibility_index": ([P, P, i64, P, P], C.c_int),
        "siting_autotune": ([P, i64, i64, i64, P, i64, P, P, i32, P, P, sz, P, P, P, i32],
                            C.c_int),
        "siting_autotune_candidates": ([i32, P, i32], C.c_int),
        "siting_greedy_workspace_size": ([i64], sz),
        "siting_greedy": ([P, P, P, i64, i64, i64, i32, i64, P, P, P, P, P, sz, P], C.c_int),
        "siting_greedy_noalloc": ([P, P, P, i64, i64, i64, i32, i64, P, P, P, P, P], C.c_int),
        "siting_greedy_parallel": ([P, P, P, i64, i64, i64, i32, i64, i32, P, P, P, P, P, sz, P],
                                   C.c_int),
        "siting_greedy_intervisible": ([P, P, P, i64, i64, i64, i32, i64, P, P, P, P, P, sz, P],
                                       C.c_int),
        "siting_cnn_param_count": ([], C.c_int),
        "siting_cnn_workspace_size": ([i64], sz),
        "siting_cnn_forward": ([P, P, i64, i64, i64, P, i64, P, P, sz, P], C.c_int),
        "siting_cnn_backward": ([P, P, i64, P, P, P, sz, P], C.c_int),
        "siting_cnn_adam": ([P, P, P, P, i64, i32, C.c_float, C.c_float, C.c_float, C.c_float, P],
                            C.c_int),
        "siting_cnn_score_terrain": ([P, P, i64, i64, i64, i32, P, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib, sig


_lib, _SIGNATURES = _load()
EXPORTED = tuple(_SIGNATURES)


def lib():
    return _lib


def last_error() -> str:
    return _lib.siting_last_error().decode()


def _check(fn: str, rc: int):
    if rc != SITING_OK:
        raise SitingError(fn, rc, last_error())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_terrain(z):
    import torch
    if not (isinstance(z, torch.Tensor) and z.is_cuda and z.dtype == torch.int16 and z.dim() == 2):
        raise TypeError("terrain must be a 2-D int16 tensor on the HIP device")
    if z.stride(1) != 1:
        raise ValueError("terrain rows must be contiguous")
    return z.shape[0], z.shape[1], z.stride(0)


def siting_abi_version() -> int:
    return int(_lib.siting_abi_version())


def siting_device_cus() -> int:
    v = C.c_int32()
    _check("siting_device_cus", _lib.siting_device_cus(C.byref(v)))
    return int(v.value)


def siting_vix(z, roi, h_t, h_r, K, seed, count=None, stream=None):
    """uint8 visible-receiver count of every post (device tensor)."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    if count is None:
        count = torch.empty((nr, nc), dtype=torch.uint8, device=z.device)
    _check("siting_vix", _lib.siting_vix(_ptr(z), nr, nc, ld, int(roi), int(h_t), int(h_r),
                                         int(K), C.c_uint64(int(seed) & (2**64 - 1)),
                                         _ptr(count), _stream(stream)))
    return count


def siting_vix_stats(z, roi, h_t, h_r, K, seed, count=None, stream=None):
    """Counting variant of siting_vix: returns (count, los_steps, los_tests,
    (lowest, highest) element offset of the terrain reads from global memory)."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    if count is None:
        count = torch.empty((nr, nc), dtype=torch.uint8, device=z.device)
    stats = torch.zeros(4, dtype=torch.int64, device=z.device)
    _check("siting_vix_stats", _lib.siting_vix_stats(
        _ptr(z), nr, nc, ld, int(roi), int(h_t), int(h_r), int(K),
        C.c_uint64(int(seed) & (2**64 - 1)), _ptr(count), _ptr(stats), _stream(stream)))
    st = stats.cpu().tolist()
    return count, int(st[0]), int(st[1]), (int(st[2]), int(st[3]))


def siting_findmax(key, z, grid_r, grid_c, k, key_stride=1, cand=None, stream=None):
    """int64 candidate post indices (grid_r*grid_c*k, -1 padded)."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    if key.dtype == torch.uint8:
        kt = SITING_KEY_U8
    elif key.dtype == torch.float32:
        kt = SITING_KEY_F32
    else:
        raise TypeError("key must be uint8 or float32")
    if not key.is_contiguous():
        raise ValueError("key must be contiguous")
    if cand is None:
        cand = torch.empty(grid_r * grid_c * k, dtype=torch.int64, device=z.device)
    _check("siting_findmax", _lib.siting_findmax(_ptr(key), kt, int(key_stride), _ptr(z), nr, nc,
                                                 ld, int(grid_r), int(grid_c), int(k), _ptr(cand),
                                                 _stream(stream)))
    return cand


def siting_viewshed_layout(obs_host: np.ndarray, nrows: int, ncols: int) -> np.ndarray:
    """Host: int64 offsets[n+1] of each observer's window bitmap (words)."""
    obs_host = np.ascontiguousarray(obs_host, OBSERVER_DTYPE)
    off = np.zeros(len(obs_host) + 1, np.int64)
    rc = _lib.siting_viewshed_layout(_ptr(obs_host), len(obs_host), int(nrows), int(ncols),
                                     _ptr(off))
    if rc < 0:
        raise SitingError("siting_viewshed_layout", int(rc), last_error())
    return off


def siting_viewshed_order(obs_host: np.ndarray) -> np.ndarray:
    """Host: processing order, longest ROI first."""
    obs_host = np.ascontiguousarray(obs_host, OBSERVER_DTYPE)
    order = np.zeros(len(obs_host), np.int32)
    _check("siting_viewshed_order", _lib.siting_viewshed_order(_ptr(obs_host), len(obs_host),
                                                               _ptr(order)))
    return order


def siting_viewshed_workspace_size() -> int:
    return int(_lib.siting_viewshed_workspace_size())


def siting_viewshed_default_schedule(rmax: int) -> Schedule:
    s = Schedule()
    _check("siting_viewshed_default_schedule",
           _lib.siting_viewshed_default_schedule(int(rmax), C.byref(s)))
    return s


def observers_to_device(obs_host: np.ndarray, device="cuda"):
    """Observer records as a device int32 tensor of shape (n, 5)."""
    import torch
    a = np.ascontiguousarray(obs_host, OBSERVER_DTYPE).view(np.int32).reshape(-1, 5)
    return torch.from_numpy(a.copy()).to(device)


def siting_viewshed_batch(z, obs_dev, offsets_dev, rmax, order_dev=None, sched=None,
                          sink=SITING_SINK_BITMAP, bitmaps=None, visible=None, cells=None,
                          ws=None, stream=None):
    """Viewsheds of all observers in one persistent launch.  Returns bitmaps
    (sink BITMAP) or (visible, cells) (sink COUNT)."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    n = obs_dev.shape[0]
    dev = z.device
    if ws is None:
        ws = torch.empty(siting_viewshed_workspace_size(), dtype=torch.uint8, device=dev)
    if sink == SITING_SINK_BITMAP and bitmaps is None:
        total = int(offsets_dev[-1].item()) if n else 0
        bitmaps = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    if sink == SITING_SINK_COUNT:
        if visible is None:
            visible = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if cells is None:
            cells = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    sp = C.byref(sched) if sched is not None else None
    _check("siting_viewshed_batch", _lib.siting_viewshed_batch(
        _ptr(z), nr, nc, ld, _ptr(obs_dev), n,
        _ptr(offsets_dev) if offsets_dev is not None else None,
        _ptr(order_dev) if order_dev is not None else None, int(rmax), sp, int(sink),
        _ptr(bitmaps) if bitmaps is not None else None,
        _ptr(visible) if sink == SITING_SINK_COUNT else None,
        _ptr(cells) if sink == SITING_SINK_COUNT else None,
        _ptr(ws), ws.numel(), _stream(stream)))
    return bitmaps if sink == SITING_SINK_BITMAP else (visible, cells)


def siting_visibility_index(visible, cells, vi=None, stream=None):
    """Exact visibility index (visible - 1) / (cells - 1) per observer from
    the count sink's device counts (float32 device tensor)."""
    import torch
    n = visible.numel()
    if cells.numel() != n:
        raise ValueError("visible and cells differ in length")
    if vi is None:
        vi = torch.empty(max(n, 1), dtype=torch.float32, device=visible.device)
    _check("siting_visibility_index", _lib.siting_visibility_index(
        _ptr(visible), _ptr(cells), n, _ptr(vi), _stream(stream)))
    return vi[:n]


def siting_viewshed_r3(z, obs_dev, offsets_dev, bitmaps=None, stream=None):
    """Exact per-cell viewsheds (every disk cell by its own line of sight) in
    the layout of siting_viewshed_batch.  Returns the bitmaps."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    n = obs_dev.shape[0]
    if bitmaps is None:
        total = int(offsets_dev[-1].item()) if n else 0
        bitmaps = torch.zeros(max(total, 1), dtype=torch.int64, device=z.device)
    _check("siting_viewshed_r3", _lib.siting_viewshed_r3(
        _ptr(z), nr, nc, ld, _ptr(obs_dev), n, _ptr(offsets_dev), _ptr(bitmaps),
        _stream(stream)))
    return bitmaps


def siting_autotune_candidates(rmax: int):
    arr = (Schedule * 64)()
    m = _lib.siting_autotune_candidates(int(rmax), arr, 64)
    if m < 0:
        raise SitingError("siting_autotune_candidates", m, last_error())
    return [arr[i] for i in range(min(m, 64))]


def siting_autotune(z, obs_dev, offsets_dev, rmax, bitmaps, order_dev=None, ws=None, stream=None):
    """Times every candidate schedule; returns (best Schedule, [ms per candidate])."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    if ws is None:
        ws = torch.empty(siting_viewshed_workspace_size(), dtype=torch.uint8, device=z.device)
    best = Schedule()
    times = (C.c_float * 64)()
    _check("siting_autotune", _lib.siting_autotune(
        _ptr(z), nr, nc, ld, _ptr(obs_dev), obs_dev.shape[0], _ptr(offsets_dev),
        _ptr(order_dev) if order_dev is not None else None, int(rmax), _ptr(bitmaps), _ptr(ws),
        ws.numel(), _stream(stream), C.byref(best), times, 64))
    n = len(siting_autotune_candidates(rmax))
    return best, [float(times[i]) for i in range(min(n, 64))]


def siting_greedy_workspace_size(n: int) -> int:
    return int(_lib.siting_greedy_workspace_size(int(n)))


def siting_greedy(bitmaps, offsets_dev, obs_dev, nrows, ncols, max_obs, target_cells,
                  cumulative=None, ws=None, stream=None, intervisible=False, parallel=0):
    """Greedy SITE.  Returns (selected, gains, nselected, cumulative) device
    tensors; selected/gains hold max_obs entries, the first nselected valid.
    intervisible=True calls siting_greedy_intervisible; parallel=m > 0 calls
    siting_greedy_parallel with batch m (synchronizes the stream)."""
    import torch
    dev = bitmaps.device
    n = obs_dev.shape[0]
    W = (ncols + 63) // 64
    if cumulative is None:
        cumulative = torch.empty((nrows, W), dtype=torch.int64, device=dev)
    selected = torch.full((max(max_obs, 1),), -1, dtype=torch.int64, device=dev)
    gains = torch.zeros((max(max_obs, 1),), dtype=torch.int64, device=dev)
    nsel = torch.zeros(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = torch.empty(max(siting_greedy_workspace_size(n), 1), dtype=torch.uint8, device=dev)
    if parallel and intervisible:
        raise ValueError("the parallel-round SITE has no intervisibility variant")
    if parallel:
        _check("siting_greedy_parallel", _lib.siting_greedy_parallel(
            _ptr(bitmaps), _ptr(offsets_dev), _ptr(obs_dev), n, int(nrows), int(ncols),
            int(max_obs), int(target_cells), int(parallel), _ptr(cumulative), _ptr(selected),
            _ptr(gains), _ptr(nsel), _ptr(ws), ws.numel(), _stream(stream)))
        return selected, gains, nsel, cumulative
    name = "siting_greedy_intervisible" if intervisible else "siting_greedy"
    _check(name, getattr(_lib, name)(
        _ptr(bitmaps), _ptr(offsets_dev), _ptr(obs_dev), n, int(nrows), int(ncols), int(max_obs),
        int(target_cells), _ptr(cumulative), _ptr(selected), _ptr(gains), _ptr(nsel), _ptr(ws),
        ws.numel(), _stream(stream)))
    return selected, gains, nsel, cumulative


SITING_GREEDY_NOALLOC_MAX_N = 1048576


def siting_greedy_noalloc(bitmaps, offsets_dev, obs_dev, nrows, ncols, max_obs, target_cells,
                          cumulative, selected, gains, nselected, stream=None):
    """Greedy SITE into caller-owned outputs (cumulative: nrows x
    ceil(ncols/64) words; selected, gains: int64[max_obs]; nselected:
    int32[1]), with the library's static workspace: nothing is allocated."""
    n = obs_dev.shape[0]
    _check("siting_greedy_noalloc", _lib.siting_greedy_noalloc(
        _ptr(bitmaps), _ptr(offsets_dev), _ptr(obs_dev), n, int(nrows), int(ncols), int(max_obs),
        int(target_cells), _ptr(cumulative), _ptr(selected), _ptr(gains), _ptr(nselected),
        _stream(stream)))
    return selected, gains, nselected, cumulative


# ---------------------------------------------------------------- CNN ------
def siting_cnn_param_count() -> int:
    return int(_lib.siting_cnn_param_count())


def siting_cnn_workspace_size(batch: int) -> int:
    return int(_lib.siting_cnn_workspace_size(int(batch)))


def cnn_workspace(batch: int, device="cuda"):
    import torch
    return torch.empty(max(siting_cnn_workspace_size(batch), 1), dtype=torch.uint8, device=device)


def siting_cnn_forward(params, z, centres, ws, pred=None, stream=None):
    """Training forward over device int64 centres; returns predictions."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    B = centres.numel()
    if pred is None:
        pred = torch.empty(B, dtype=torch.float32, device=z.device)
    _check("siting_cnn_forward", _lib.siting_cnn_forward(
        _ptr(params), _ptr(z), nr, nc, ld, _ptr(centres), B, _ptr(pred), _ptr(ws), ws.numel(),
        _stream(stream)))
    return pred


def siting_cnn_backward(params, labels, ws, grad=None, loss=None, stream=None):
    """Gradient of the MSE loss for the last forward on ws: (grad, loss)."""
    import torch
    B = labels.numel()
    if grad is None:
        grad = torch.empty(siting_cnn_param_count(), dtype=torch.float32, device=labels.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=labels.device)
    _check("siting_cnn_backward", _lib.siting_cnn_backward(
        _ptr(params), _ptr(labels), B, _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
        _stream(stream)))
    return grad, loss


def siting_cnn_adam(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check("siting_cnn_adam", _lib.siting_cnn_adam(
        _ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(), int(step), float(lr),
        float(beta1), float(beta2), float(eps), _stream(stream)))


def siting_cnn_score_terrain(params, z, stride, score=None, stream=None):
    """Predicted visibility index on the stride lattice (device float32
    tensor of ceil(nrows/stride) x ceil(ncols/stride))."""
    import torch
    nr, nc, ld = _dev_terrain(z)
    if score is None:
        score = torch.empty(((nr + stride - 1) // stride, (nc + stride - 1) // stride),
                            dtype=torch.float32, device=z.device)
    _check("siting_cnn_score_terrain", _lib.siting_cnn_score_terrain(
        _ptr(params), _ptr(z), nr, nc, ld, int(stride), _ptr(score), _stream(stream)))
    return score
