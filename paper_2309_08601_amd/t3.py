"""Thin ctypes binding of the t3pcf C ABI (include/t3pcf.h).

Argument marshalling only: every step of the estimator runs in the HIP
library.  PyTorch provides device memory and the current stream.  If the
library is not built this module raises on import; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libt3pcf.so")

T3_OK = 0
T3_EINVAL = -1
T3_ERANGE = -2
T3_ENOMEM = -3
T3_EHIP = -4
T3_ELATTICE = -5
GRID_METHODS = {"auto": 0, "direct": 1, "fft": 2}

PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp16x3": 2, "bf16x6": 3}
T3_FLAG_KEEP_JK = 1
T3_FLAG_TIMING = 2
T3_FLAG_NO_GRAPH = 4
T3_FLAG_EDGE_CORRECT = 8
T3_FLAG_NO_LANE = 16
T3_FLAG_KEEP_PLANES = 32
T3_FLAG_DETERMINISTIC = 64


class t3_params(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("edges", ctypes.POINTER(ctypes.c_double)),
                ("n_max", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("lattice_unit", ctypes.c_double), ("box_lo_x", ctypes.c_int32),
                ("box_lo_y", ctypes.c_int32), ("box_size", ctypes.c_int64),
                ("cell_arcmin", ctypes.c_double), ("chunk_centres", ctypes.c_int32),
                ("scan_mode", ctypes.c_int32), ("max_workspace_bytes", ctypes.c_int64),
                ("lane_neighbours", ctypes.c_double), ("tile_mode", ctypes.c_int32)]


class t3_catalog(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("g1", ctypes.c_void_p), ("g2", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class t3_sphere_catalog(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ra", ctypes.c_void_p), ("dec", ctypes.c_void_p),
                ("g1", ctypes.c_void_p), ("g2", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class t3_patch(ctypes.Structure):
    _fields_ = [("ra_lo", ctypes.c_double), ("ra_hi", ctypes.c_double), ("dec_lo", ctypes.c_double),
                ("dec_hi", ctypes.c_double)]


class T3Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"t3pcf error {code}: {msg}")
        self.code = code


EXPORTED = ["t3_plan_create", "t3_plan_destroy", "t3_forward", "t3_forward_tomo", "t3_harmonics",
            "t3_normalise_resum", "t3_normalise_backward", "t3_backward", "t3_autotune", "t3_stage_times",
            "t3_workspace_bytes", "t3_graph_stats", "t3_plan_settings", "t3_forward_noalloc", "t3_error_string",
            "t3_last_error_message", "t3_version"]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"t3pcf HIP library not built: {path} (run paper_2309_08601_amd/build.py)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.t3_plan_create.argtypes = [P(t3_params), P(vp)]
    lib.t3_plan_create.restype = ctypes.c_int
    lib.t3_plan_destroy.argtypes = [vp]
    lib.t3_plan_destroy.restype = None
    lib.t3_forward.argtypes = [vp, P(t3_catalog), vp, ctypes.c_int64, vp, P(ctypes.c_int64), vp]
    lib.t3_forward.restype = ctypes.c_int
    lib.t3_forward_noalloc.argtypes = [vp, P(t3_catalog), vp, ctypes.c_int64, vp, P(ctypes.c_int64), vp]
    lib.t3_forward_noalloc.restype = ctypes.c_int
    lib.t3_forward_tomo.argtypes = [vp, P(t3_catalog), ctypes.c_int32, P(vp), P(ctypes.c_int64), vp,
                                    P(ctypes.c_int64), vp]
    lib.t3_forward_tomo.restype = ctypes.c_int
    lib.t3_forward_sphere.argtypes = [vp, P(t3_sphere_catalog), P(t3_patch), ctypes.c_int32, ctypes.c_double, vp,
                                      P(ctypes.c_int64), vp]
    lib.t3_forward_sphere.restype = ctypes.c_int
    lib.t3_forward_grid.argtypes = [vp, P(t3_catalog), ctypes.c_int64, P(ctypes.c_int32), ctypes.c_int32, vp,
                                    P(ctypes.c_int64), vp]
    lib.t3_forward_grid.restype = ctypes.c_int
    lib.t3_harmonics.argtypes = [vp, P(t3_catalog), vp, ctypes.c_int64, vp, vp, vp, vp]
    lib.t3_harmonics.restype = ctypes.c_int
    lib.t3_normalise_resum.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    lib.t3_normalise_resum.restype = ctypes.c_int
    lib.t3_x_to_centroid.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double), vp, vp]
    lib.t3_x_to_centroid.restype = ctypes.c_int
    lib.t3_aperture_stats.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32,
                                      vp, vp, vp]
    lib.t3_aperture_stats.restype = ctypes.c_int
    lib.t3_normalise_backward.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    lib.t3_normalise_backward.restype = ctypes.c_int
    lib.t3_backward.argtypes = [vp, P(t3_catalog), vp, ctypes.c_int64, vp, vp, vp, vp, vp]
    lib.t3_backward.restype = ctypes.c_int
    lib.t3_autotune.argtypes = [vp, P(t3_catalog), ctypes.c_int32, ctypes.c_int64, P(ctypes.c_double), vp]
    lib.t3_autotune.restype = ctypes.c_int
    lib.t3_stage_times.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
    lib.t3_stage_times.restype = ctypes.c_int
    lib.t3_workspace_bytes.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64)]
    lib.t3_workspace_bytes.restype = ctypes.c_int
    lib.t3_graph_stats.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64)]
    lib.t3_graph_stats.restype = ctypes.c_int
    lib.t3_plan_settings.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_double),
                                     P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.t3_plan_settings.restype = ctypes.c_int
    lib.t3_error_string.argtypes = [ctypes.c_int]
    lib.t3_error_string.restype = ctypes.c_char_p
    lib.t3_last_error_message.argtypes = []
    lib.t3_last_error_message.restype = ctypes.c_char_p
    lib.t3_version.argtypes = []
    lib.t3_version.restype = ctypes.c_char_p
    return lib


_lib = load_library()


def _check(rc: int):
    if rc != T3_OK:
        raise T3Error(rc, _lib.t3_last_error_message().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class DeviceCatalog:
    """Device-resident SoA catalog (int32 lattice positions, float32 shears)."""

    def __init__(self, x, y, g1, g2, w, device="cuda"):
        def t(a, dt):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device).contiguous()
        self.x = t(x, torch.int32)
        self.y = t(y, torch.int32)
        self.g1 = t(g1, torch.float32)
        self.g2 = t(g2, torch.float32)
        self.w = t(w, torch.float32)
        self.n = int(self.x.shape[0])

    @classmethod
    def from_catalog(cls, cat, device="cuda"):
        return cls(cat.x, cat.y, cat.g1, cat.g2, cat.w, device=device)

    def c_struct(self) -> t3_catalog:
        return t3_catalog(self.n, self.x.data_ptr(), self.y.data_ptr(), self.g1.data_ptr(),
                          self.g2.data_ptr(), self.w.data_ptr())


def grid_levels(edges: Sequence[float], delta_arcmin: float, min_ratio: float = 20.0,
                theta_disc: float = 0.0, max_level: int = 8) -> List[int]:
    """Level of each radial bin for the combined estimator: 0 (discrete)
    while the bin's lower edge is below theta_disc, else the coarsest grid
    whose pixel Delta_l = delta_arcmin 2^(l-1) satisfies lower edge >=
    min_ratio Delta_l (Sect. 3.3: agreement at the sub-per-cent level for
    Theta >= 20 Delta); 0 if no grid qualifies.  Non-decreasing."""
    out: List[int] = []
    for lo in list(edges)[:-1]:
        lvl = 0
        if lo >= theta_disc:
            while lvl < max_level and lo >= min_ratio * delta_arcmin * 2.0 ** lvl:
                lvl += 1
        out.append(max(lvl, out[-1]) if out else lvl)
    return out


class Plan:
    """Owns one t3_plan (radial bins, n_max, precision, lattice box)."""

    def __init__(self, edges: Sequence[float], n_max: int, box_lo=(0, 0), box_size: int = 1 << 30,
                 precision: str = "fp32", keep_jk: bool = False, lattice_unit: float = 0.0,
                 cell_arcmin: float = 0.0, chunk_centres: int = 0, timing: bool = False,
                 graph: bool = True, scan_mode: int = 0, edge_correct: bool = False, lane: bool = True,
                 keep_planes: bool = False, deterministic: bool = False, max_workspace_bytes: int = 0,
                 lane_neighbours: float = 0.0, tile_mode: int = 0):
        self.edges = np.ascontiguousarray(edges, dtype=np.float64)
        self.B = len(self.edges) - 1
        self.n_max = int(n_max)
        self.edge_correct = bool(edge_correct)
        self.w_max = 2 * self.n_max if self.edge_correct else self.n_max
        p = t3_params(self.B, self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.n_max,
                      PRECISIONS[precision],
                      (T3_FLAG_KEEP_JK if keep_jk else 0) | (T3_FLAG_TIMING if timing else 0)
                      | (0 if graph else T3_FLAG_NO_GRAPH) | (T3_FLAG_EDGE_CORRECT if edge_correct else 0)
                      | (0 if lane else T3_FLAG_NO_LANE) | (T3_FLAG_KEEP_PLANES if keep_planes else 0)
                      | (T3_FLAG_DETERMINISTIC if deterministic else 0),
                      float(lattice_unit),
                      int(box_lo[0]), int(box_lo[1]), int(box_size), float(cell_arcmin),
                      int(chunk_centres), int(scan_mode), int(max_workspace_bytes), float(lane_neighbours),
                      int(tile_mode))
        h = ctypes.c_void_p()
        _check(_lib.t3_plan_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.t3_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out_shape(self, sets: int = 1):
        if self.edge_correct:  # Upsilon blocks then N_0..N_{2 n_max}
            return (sets, 4 * (self.n_max + 1) + self.w_max + 1, self.B, self.B, 2)
        return (sets, 5, self.n_max + 1, self.B, self.B, 2)

    def _trail(self) -> int:
        return len(self._out_shape()) - 1  # trailing dims of one set (real view)

    def split_ups(self, ups: torch.Tensor):
        """(Upsilon [..., 4, n_max+1, B, B], N [..., w_max+1, B, B]) of a
        forward output (complex)."""
        nm, B = self.n_max, self.B
        if not self.edge_correct:
            return ups[..., :4, :, :, :], ups[..., 4, :, :, :]
        lead = ups.shape[:-3]
        u4 = ups[..., :4 * (nm + 1), :, :].reshape(lead + (4, nm + 1, B, B))
        return u4, ups[..., 4 * (nm + 1):, :, :]

    def forward(self, cat: DeviceCatalog, centres: Optional[torch.Tensor] = None,
                out: Optional[torch.Tensor] = None):
        """Upsilon_{0..3,n} and N_n for n = 0..n_max: complex128 [5, n_max+1, B, B]."""
        if out is None:
            out = torch.empty(self._out_shape()[1:], dtype=torch.float64, device=cat.x.device)
        cs = cat.c_struct()
        npairs = ctypes.c_int64(0)
        if centres is not None:
            centres = centres.to(torch.int32).contiguous()
        _check(_lib.t3_forward(self._h, ctypes.byref(cs), _ptr(centres),
                               -1 if centres is None else int(centres.numel()), _ptr(out),
                               ctypes.byref(npairs), _stream()))
        return torch.view_as_complex(out), int(npairs.value)

    def forward_noalloc(self, cat: DeviceCatalog, centres: Optional[torch.Tensor] = None,
                        out: Optional[torch.Tensor] = None):
        """forward() with every internal buffer in the library's static device
        scratch (nothing allocated by the library; `out` may be preallocated
        by the caller)."""
        if out is None:
            out = torch.empty(self._out_shape()[1:], dtype=torch.float64, device=cat.x.device)
        cs = cat.c_struct()
        npairs = ctypes.c_int64(0)
        if centres is not None:
            centres = centres.to(torch.int32).contiguous()
        _check(_lib.t3_forward_noalloc(self._h, ctypes.byref(cs), _ptr(centres),
                                       -1 if centres is None else int(centres.numel()), _ptr(out),
                                       ctypes.byref(npairs), _stream()))
        return torch.view_as_complex(out), int(npairs.value)

    def forward_tomo(self, cats: List[DeviceCatalog], centres: Optional[List[Optional[torch.Tensor]]] = None,
                     out: Optional[torch.Tensor] = None):
        nz = len(cats)
        if out is None:
            out = torch.empty((nz, nz, nz) + self._out_shape()[1:], dtype=torch.float64,
                              device=cats[0].x.device)
        arr = (t3_catalog * nz)(*[c.c_struct() for c in cats])
        cptr = None
        cnt = None
        keep = []
        if centres is not None:
            cptr = (ctypes.c_void_p * nz)()
            cnt = (ctypes.c_int64 * nz)()
            for z, c in enumerate(centres):
                if c is None:
                    cptr[z] = None
                    cnt[z] = -1
                else:
                    c = c.to(torch.int32).contiguous()
                    keep.append(c)
                    cptr[z] = c.data_ptr()
                    cnt[z] = c.numel()
        npairs = ctypes.c_int64(0)
        _check(_lib.t3_forward_tomo(self._h, arr, nz, cptr, cnt, _ptr(out), ctypes.byref(npairs),
                                    _stream()))
        return torch.view_as_complex(out), int(npairs.value)

    def forward_sphere(self, ra: torch.Tensor, dec: torch.Tensor, g1: torch.Tensor, g2: torch.Tensor,
                       w: torch.Tensor, patches, theta_max: float, out: Optional[torch.Tensor] = None):
        """Curved-sky catalog (device tensors: ra, dec float64 degrees; g1, g2,
        w float32) through flat patches [(ra_lo, ra_hi, dec_lo, dec_hi), ...]
        with theta_max (arcmin) overlap; multipoles summed over patches."""
        arrs = [ra.to(torch.float64).contiguous(), dec.to(torch.float64).contiguous(),
                g1.to(torch.float32).contiguous(), g2.to(torch.float32).contiguous(),
                w.to(torch.float32).contiguous()]
        cs = t3_sphere_catalog(int(arrs[0].numel()), *[a.data_ptr() for a in arrs])
        pa = (t3_patch * len(patches))(*[t3_patch(*map(float, p)) for p in patches])
        if out is None:
            out = torch.empty(self._out_shape()[1:], dtype=torch.float64, device=arrs[0].device)
        npairs = ctypes.c_int64(0)
        _check(_lib.t3_forward_sphere(self._h, ctypes.byref(cs), pa, len(patches), float(theta_max), _ptr(out),
                                      ctypes.byref(npairs), _stream()))
        return torch.view_as_complex(out), int(npairs.value)

    def forward_grid(self, cat: DeviceCatalog, delta: int, levels: Sequence[int], method: str = "auto",
                     out: Optional[torch.Tensor] = None):
        """Combined discrete / grid-based multipoles: levels[b] = 0 for a
        discrete bin, l >= 1 for pixels of side delta * 2^(l-1) lattice steps
        (non-decreasing in b); method "direct", "fft" or "auto" per level.
        Same output as forward."""
        if len(levels) != self.B:
            raise ValueError("one level per radial bin")
        lv = (ctypes.c_int32 * self.B)(*[int(v) for v in levels])
        if out is None:
            out = torch.empty(self._out_shape()[1:], dtype=torch.float64, device=cat.x.device)
        cs = cat.c_struct()
        npairs = ctypes.c_int64(0)
        _check(_lib.t3_forward_grid(self._h, ctypes.byref(cs), int(delta), lv, GRID_METHODS[method], _ptr(out),
                                    ctypes.byref(npairs), _stream()))
        return torch.view_as_complex(out), int(npairs.value)

    def harmonics(self, cat: DeviceCatalog, centres: torch.Tensor):
        """Stage-1 sums: G [n_c, B, 2 n_max + 3] (m = -n_max-3 .. n_max-1),
        W [n_c, B, n_max + 1], D [n_c, B, 4] (complex64)."""
        centres = centres.to(torch.int32).contiguous()
        nc = int(centres.numel())
        dev = cat.x.device
        G = torch.empty((nc, self.B, 2 * self.n_max + 3, 2), dtype=torch.float32, device=dev)
        W = torch.empty((nc, self.B, self.n_max + 1, 2), dtype=torch.float32, device=dev)
        D = torch.empty((nc, self.B, 4, 2), dtype=torch.float32, device=dev)
        cs = cat.c_struct()
        _check(_lib.t3_harmonics(self._h, ctypes.byref(cs), _ptr(centres), nc, _ptr(G), _ptr(W),
                                 _ptr(D), _stream()))
        return torch.view_as_complex(G), torch.view_as_complex(W), torch.view_as_complex(D)

    def normalise_resum(self, ups: torch.Tensor, n_phi: int = 32, with_phi: bool = True):
        """Gamma_{mu,n} = Upsilon/N_0 [.., 4, n_max+1, B, B] and the resummed
        Gamma(b1, b2, Phi_k) [.., 4, B, B, n_phi] (complex128)."""
        u = torch.view_as_real(ups).contiguous() if ups.is_complex() else ups.contiguous()
        lead = u.shape[:-self._trail()]
        sets = int(np.prod(lead)) if len(lead) else 1
        gn = torch.empty(lead + (4, self.n_max + 1, self.B, self.B, 2), dtype=torch.float64,
                         device=u.device)
        gp = None
        if with_phi:
            gp = torch.empty(lead + (4, self.B, self.B, n_phi, 2), dtype=torch.float64, device=u.device)
        _check(_lib.t3_normalise_resum(self._h, _ptr(u), sets, int(n_phi), _ptr(gn), _ptr(gp), _stream()))
        return torch.view_as_complex(gn), (None if gp is None else torch.view_as_complex(gp))

    def x_to_centroid(self, gamma_phi: torch.Tensor, theta: Optional[Sequence[float]] = None) -> torch.Tensor:
        """x -> centroid projection of a resummed Gamma [..., 4, B, B, n_phi]
        (complex128), factors at (theta[b1], theta[b2], angular-bin centre);
        theta defaults to the radial bin centres."""
        g = torch.view_as_real(gamma_phi).contiguous() if gamma_phi.is_complex() else gamma_phi.contiguous()
        n_phi = int(g.shape[-2])
        lead = g.shape[:-5]
        sets = int(np.prod(lead)) if len(lead) else 1
        out = torch.empty_like(g)
        th = None
        keep = None
        if theta is not None:
            keep = np.ascontiguousarray(theta, dtype=np.float64)
            if keep.shape != (self.B,):
                raise ValueError("theta needs one radius per bin")
            th = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(_lib.t3_x_to_centroid(self._h, _ptr(g), sets, n_phi, th, _ptr(out), _stream()))
        return torch.view_as_complex(out)

    def aperture_stats(self, gamma_cent: torch.Tensor, apertures):
        """Correlators [..., n_ap, 4] (complex128: <M^3>, <M* M^2>, <M M* M>,
        <M^2 M*>) and statistics [..., n_ap, 8] (<Map^3>, <Mx Map^2>,
        <Map Mx Map>, <Map^2 Mx>, <Map Mx^2>, <Mx Map Mx>, <Mx^2 Map>, <Mx^3>)
        from a centroid-projected Gamma [..., 4, B, B, n_phi]; apertures
        [n_ap, 3] radii in arcmin."""
        g = torch.view_as_real(gamma_cent).contiguous() if gamma_cent.is_complex() else gamma_cent.contiguous()
        n_phi = int(g.shape[-2])
        lead = g.shape[:-5]
        sets = int(np.prod(lead)) if len(lead) else 1
        ap = np.ascontiguousarray(apertures, dtype=np.float64).reshape(-1, 3)
        corr = torch.empty(lead + (ap.shape[0], 4, 2), dtype=torch.float64, device=g.device)
        stats = torch.empty(lead + (ap.shape[0], 8), dtype=torch.float64, device=g.device)
        _check(_lib.t3_aperture_stats(self._h, _ptr(g), sets, n_phi,
                                      ap.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ap.shape[0],
                                      _ptr(corr), _ptr(stats), _stream()))
        return torch.view_as_complex(corr), stats

    def normalise_backward(self, ups: torch.Tensor, grad_gamma_n: torch.Tensor) -> torch.Tensor:
        """dL/dUpsilon (and dL/dN_0) from dL/dGamma_n; real views [..., 2]."""
        u = torch.view_as_real(ups).contiguous() if ups.is_complex() else ups.contiguous()
        g = torch.view_as_real(grad_gamma_n).contiguous() if grad_gamma_n.is_complex() else grad_gamma_n.contiguous()
        lead = u.shape[:-5]
        sets = int(np.prod(lead)) if len(lead) else 1
        out = torch.empty_like(u)
        _check(_lib.t3_normalise_backward(self._h, _ptr(u), sets, _ptr(g), _ptr(out), _stream()))
        return out

    def autotune(self, cats, sample_per_bin: int = 20000) -> float:
        """Pick cell size, stage-1 launch mode, lane-kernel threshold, stage-2
        tile shape and chunk capacity by timing a centre sample (cached per
        problem shape); returns the best sample time in ms (0 if cached)."""
        cats = cats if isinstance(cats, (list, tuple)) else [cats]
        arr = (t3_catalog * len(cats))(*[c.c_struct() for c in cats])
        best = ctypes.c_double(0.0)
        _check(_lib.t3_autotune(self._h, arr, len(cats), int(sample_per_bin), ctypes.byref(best), _stream()))
        return float(best.value)

    def stage_times(self):
        """(ms[4], launches[4]) of the last forward call (timing plans only):
        cell build, stage 1, stage 2, unused."""
        ms = (ctypes.c_double * 4)()
        nl = (ctypes.c_int64 * 4)()
        _check(_lib.t3_stage_times(self._h, ms, nl))
        return list(ms), list(nl)

    def settings(self) -> dict:
        """The plan's tunable settings (see t3_plan_settings)."""
        cell = ctypes.c_double(0.0)
        mode = ctypes.c_int32(0)
        lane = ctypes.c_double(0.0)
        tile = ctypes.c_int32(0)
        chunk = ctypes.c_int32(0)
        _check(_lib.t3_plan_settings(self._h, ctypes.byref(cell), ctypes.byref(mode), ctypes.byref(lane),
                                     ctypes.byref(tile), ctypes.byref(chunk)))
        return {"cell_arcmin": cell.value, "scan_mode": mode.value, "lane_neighbours": lane.value,
                "tile_mode": tile.value, "chunk_centres": chunk.value}

    def graph_stats(self):
        """(captures, launches) of the plan's chunk-schedule graph."""
        cap = ctypes.c_int64(0)
        lau = ctypes.c_int64(0)
        _check(_lib.t3_graph_stats(self._h, ctypes.byref(cap), ctypes.byref(lau)))
        return int(cap.value), int(lau.value)

    def workspace_bytes(self):
        """(in use, peak) device bytes held by the plan."""
        used = ctypes.c_int64(0)
        peak = ctypes.c_int64(0)
        _check(_lib.t3_workspace_bytes(self._h, ctypes.byref(used), ctypes.byref(peak)))
        return int(used.value), int(peak.value)

    def backward(self, cat: DeviceCatalog, grad_ups: torch.Tensor, centres: Optional[torch.Tensor] = None):
        """dL/d(g1, g2, w) of every galaxy from dL/dUpsilon (real view [..., 2]);
        centres: the forward pass's centre list (None: every galaxy)."""
        g = torch.view_as_real(grad_ups).contiguous() if grad_ups.is_complex() else grad_ups.contiguous()
        dev = cat.x.device
        gg1 = torch.empty(cat.n, dtype=torch.float32, device=dev)
        gg2 = torch.empty(cat.n, dtype=torch.float32, device=dev)
        gw = torch.empty(cat.n, dtype=torch.float32, device=dev)
        cs = cat.c_struct()
        if centres is not None:
            centres = centres.to(torch.int32).contiguous()
        _check(_lib.t3_backward(self._h, ctypes.byref(cs), _ptr(centres),
                                -1 if centres is None else int(centres.numel()), _ptr(g), _ptr(gg1), _ptr(gg2),
                                _ptr(gw), _stream()))
        return gg1, gg2, gw


def version() -> str:
    return _lib.t3_version().decode()


class GammaMultipoles(torch.autograd.Function):
    """Gamma_{mu,n}(b1, b2) = Upsilon_{mu,n} / N_0 (mu = 0..3, n = 0..n_max) as a
    differentiable function of every galaxy's (g1, g2, w), returned as a real
    view [4, n_max + 1, B, B, 2].  Forward and backward both run in the HIP
    library (t3_forward + t3_normalise_resum, t3_normalise_backward +
    t3_backward); positions are constants."""

    @staticmethod
    def forward(ctx, g1, g2, w, x, y, plan):
        cat = DeviceCatalog.__new__(DeviceCatalog)
        cat.x, cat.y = x.contiguous(), y.contiguous()
        cat.g1, cat.g2, cat.w = g1.detach().contiguous(), g2.detach().contiguous(), w.detach().contiguous()
        cat.n = int(x.shape[0])
        ups, _ = plan.forward(cat)
        gn, _ = plan.normalise_resum(ups, with_phi=False)
        ctx.plan = plan
        # the inputs go through save_for_backward so that autograd's version
        # check raises if any of them is modified in place before backward
        # (the adjoint reads them again, and kept planes must match them)
        ctx.save_for_backward(torch.view_as_real(ups), g1, g2, w, x, y)
        return torch.view_as_real(gn).clone()

    @staticmethod
    def backward(ctx, grad_out):
        ups, g1, g2, w, x, y = ctx.saved_tensors
        cat = DeviceCatalog.__new__(DeviceCatalog)
        cat.x, cat.y = x.contiguous(), y.contiguous()
        cat.g1, cat.g2, cat.w = g1.detach().contiguous(), g2.detach().contiguous(), w.detach().contiguous()
        cat.n = int(x.shape[0])
        gups = ctx.plan.normalise_backward(ups, grad_out.contiguous())
        gg1, gg2, gw = ctx.plan.backward(cat, gups)
        return gg1, gg2, gw, None, None, None
