"""Python binding of libpm: argument marshalling around the C ABI (include/pm.h).

Every step of the particle-mesh path runs in libpm's HIP kernels; this module only
allocates device tensors with torch, fills the C structs and checks status codes.
Functions keep the names of the C entry points (pm_encode -> PMContext.encode, ...).
"""

from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import PM_COMPRESSED, PM_FLOAT, PmConfig, PmSpecies, check

G_UNIT = 1.0 / (4.0 * math.pi)  # 4 pi G = 1


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


@dataclass
class FloatSpecies:
    x: torch.Tensor  # float32 [n, 3] on the device
    v: torch.Tensor
    mass: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def c(self) -> PmSpecies:
        s = PmSpecies()
        s.layout = PM_FLOAT
        s.n = self.n
        s.mass = self.mass
        s.x = _ptr(self.x)
        s.v = _ptr(self.v)
        return s


def widths_word(pos_bytes: int = 1, vel_bytes: int = 2) -> int:
    """pm_species.widths: 0 for 1-byte positions and 2-byte velocities, else P | V << 8."""
    if pos_bytes not in (1, 2) or vel_bytes not in (1, 2):
        raise ValueError("code widths are 1 or 2 bytes")
    return 0 if (pos_bytes, vel_bytes) == (1, 2) else pos_bytes | (vel_bytes << 8)


@dataclass
class CompressedSpecies:
    count: torch.Tensor  # uint8 [n_cell^3]
    pos: torch.Tensor    # [n, 3]: uint8 (1-byte codes) or int16 holding uint16 codes
    vel: torch.Tensor    # [n, 3]: int16 holding uint16 codes, or uint8 (1-byte codes)
    esc: torch.Tensor    # int64 [cap, 2] holding uint64 (cell, count)
    hdr: torch.Tensor    # uint8 [32]: pm_shdr
    mass: float
    widths: int = 0      # pm_species.widths (widths_word)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def pos_bytes(self) -> int:
        return 1 if self.widths == 0 else self.widths & 255

    @property
    def vel_bytes(self) -> int:
        return 2 if self.widths == 0 else self.widths >> 8

    def c(self) -> PmSpecies:
        s = PmSpecies()
        s.layout = PM_COMPRESSED
        s.widths = self.widths
        s.n = self.n
        s.mass = self.mass
        s.count = _ptr(self.count)
        s.pos = _ptr(self.pos)
        s.vel = _ptr(self.vel)
        s.esc = _ptr(self.esc)
        s.cap_esc = int(self.esc.shape[0])
        s.hdr = _ptr(self.hdr)
        return s

    def header(self) -> dict:
        h = self.hdr.cpu().numpy().tobytes()
        v_max, j_min, j_max, flags, n_esc, _ = np_struct_unpack(h)
        return {"v_max": np.float32(v_max), "j_min": j_min, "j_max": j_max, "flags": flags,
                "n_esc": n_esc}


def np_struct_unpack(h: bytes):
    import struct
    return struct.unpack("<fiiiqq", h)


def _species_array(species):
    arr = (PmSpecies * len(species))()
    for i, s in enumerate(species):
        arr[i] = s.c()
    return arr


class PMContext:
    """A libpm context: one mesh size, one compression-cell size, one HIP stream."""

    KERNEL_FULL, KERNEL_LONG, KERNEL_SHORT = 0, 1, 2

    def __init__(self, n_mesh: int, n_cell: int, brick: int | None = None,
                 G: float = G_UNIT, soft_cells: float = 1.0, device: str = "cuda",
                 box: float = 1.0, kernel: int = 0, r_split: float = 0.0):
        self.lib = _lib.lib()
        dev = torch.device(device)
        if dev.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("libpm needs a ROCm GPU (torch.cuda unavailable)")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        torch.cuda.set_device(self.device)
        if brick is None:
            brick = self.default_brick(n_mesh, n_cell)
        self.n_mesh, self.n_cell, self.brick = n_mesh, n_cell, brick
        self.G, self.soft_cells, self.box = G, soft_cells, float(box)
        self.kernel, self.r_split = int(kernel), float(r_split)
        cfg = PmConfig(n_mesh, n_cell, brick, 0, float(box), G, soft_cells, int(kernel), 0,
                       float(r_split))
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(self.lib.pm_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h)), "pm_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.pm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def default_brick(n_mesh: int, n_cell: int) -> int:
        """Cells per brick side: 16 mesh nodes per brick side where the cells allow."""
        return max(1, min(8, n_cell, 16 // max(1, n_mesh // n_cell)))

    @staticmethod
    def query_sizes(n_mesh: int, n_cell: int, brick: int, n_max: int, n_sp: int,
                    box: float = 1.0) -> dict:
        """pm_query_sizes: device bytes of a configuration (no GPU needed)."""
        lib = _lib.lib()
        cfg = PmConfig(n_mesh, n_cell, brick, 0, float(box), G_UNIT, 1.0, 0, 0, 0.0)
        out = _lib.PmSizes()
        check(lib.pm_query_sizes(ctypes.byref(cfg), int(n_max), int(n_sp), ctypes.byref(out)),
              "pm_query_sizes")
        return {name: getattr(out, name) for name, _ in _lib.PmSizes._fields_}

    def scratch_bytes(self) -> int:
        v = ctypes.c_int64()
        check(self.lib.pm_scratch_bytes(self.h, ctypes.byref(v)), "pm_scratch_bytes")
        return v.value

    # ----------------------------------------------------------- allocation --
    def float_species(self, x, v, mass: float) -> FloatSpecies:
        x = torch.as_tensor(x, dtype=torch.float32).to(self.device).contiguous()
        v = torch.as_tensor(v, dtype=torch.float32).to(self.device).contiguous()
        return FloatSpecies(x.reshape(-1, 3), v.reshape(-1, 3), float(mass))

    def empty_compressed(self, n: int, mass: float, cap_esc: int | None = None,
                         widths: int = 0) -> CompressedSpecies:
        if cap_esc is None:
            cap_esc = max(16, n // 255 + 1)
        d = self.device
        pb = 1 if widths == 0 else widths & 255
        vb = 2 if widths == 0 else widths >> 8
        return CompressedSpecies(
            count=torch.empty(self.n_cell ** 3, dtype=torch.uint8, device=d),
            pos=torch.empty((n, 3), dtype=torch.uint8 if pb == 1 else torch.int16, device=d),
            vel=torch.empty((n, 3), dtype=torch.int16 if vb == 2 else torch.uint8, device=d),
            esc=torch.zeros((cap_esc, 2), dtype=torch.int64, device=d),
            hdr=torch.zeros(32, dtype=torch.uint8, device=d),
            mass=float(mass), widths=int(widths))

    def empty_like(self, s):
        if isinstance(s, FloatSpecies):
            return FloatSpecies(torch.empty_like(s.x), torch.empty_like(s.v), s.mass)
        return self.empty_compressed(s.n, s.mass, int(s.esc.shape[0]), s.widths)

    # ------------------------------------------------------------ the calls --
    def sync(self):
        check(self.lib.pm_sync(self.h), "pm_sync")

    def last_error_detail(self) -> int:
        v = ctypes.c_int64()
        check(self.lib.pm_last_error_detail(self.h, ctypes.byref(v)), "pm_last_error_detail")
        return v.value

    def encode(self, fs: FloatSpecies, want_perm: bool = False, cap_esc: int | None = None,
               widths: int = 0):
        """pm_encode; widths: code widths of the result (widths_word)."""
        out = self.empty_compressed(fs.n, fs.mass, cap_esc, widths)
        perm = torch.empty(fs.n, dtype=torch.int64, device=self.device) if want_perm else None
        a, b = fs.c(), out.c()
        check(self.lib.pm_encode(self.h, ctypes.byref(a), ctypes.byref(b), _ptr(perm)),
              "pm_encode")
        return (out, perm) if want_perm else out

    def decode(self, cs: CompressedSpecies) -> FloatSpecies:
        out = FloatSpecies(torch.empty((cs.n, 3), dtype=torch.float32, device=self.device),
                           torch.empty((cs.n, 3), dtype=torch.float32, device=self.device),
                           cs.mass)
        a, b = cs.c(), out.c()
        check(self.lib.pm_decode(self.h, ctypes.byref(a), ctypes.byref(b)), "pm_decode")
        return out

    def deposit(self, species, rho: torch.Tensor | None = None) -> torch.Tensor:
        n = self.n_mesh
        if rho is None:
            rho = torch.empty((n, n, n), dtype=torch.float32, device=self.device)
        arr = _species_array(species)
        check(self.lib.pm_deposit(self.h, arr, len(species), _ptr(rho)), "pm_deposit")
        return rho

    def force(self, rho: torch.Tensor, acc: torch.Tensor | None = None,
              a_max: torch.Tensor | None = None):
        """Acceleration mesh [3, n, n, n] and max |a| (device float tensor)."""
        n = self.n_mesh
        if acc is None:
            acc = torch.empty((3, n, n, n), dtype=torch.float32, device=self.device)
        if a_max is None:
            a_max = torch.zeros(1, dtype=torch.float32, device=self.device)
        check(self.lib.pm_force(self.h, _ptr(rho), _ptr(acc), _ptr(a_max)), "pm_force")
        return acc, a_max

    def kick_drift(self, species, acc, a_max, c_kick: float, c_drift: float, out=None):
        if out is None:
            out = [self.empty_like(s) for s in species]
        a, b = _species_array(species), _species_array(out)
        check(self.lib.pm_kick_drift(self.h, a, b, len(species), _ptr(acc), _ptr(a_max),
                                     float(c_kick), float(c_drift)), "pm_kick_drift")
        return out

    def kick_drift_perm(self, species, acc, a_max, c_kick: float, c_drift: float, out=None):
        """kick_drift plus, per species, new stream position -> old stream position."""
        if out is None:
            out = [self.empty_like(s) for s in species]
        perms = [torch.empty(s.n, dtype=torch.int64, device=self.device) for s in species]
        a, b = _species_array(species), _species_array(out)
        pp = (ctypes.c_void_p * len(species))(*[_ptr(p) for p in perms])
        check(self.lib.pm_kick_drift_perm(self.h, a, b, len(species), _ptr(acc), _ptr(a_max),
                                          float(c_kick), float(c_drift), pp),
              "pm_kick_drift_perm")
        return out, perms

    def step(self, species, dt: float, out=None):
        if out is None:
            out = [self.empty_like(s) for s in species]
        a, b = _species_array(species), _species_array(out)
        check(self.lib.pm_step(self.h, a, b, len(species), float(dt)), "pm_step")
        return out

    def pp_accel(self, species, r_soft: float, app_max: torch.Tensor | None = None):
        """pm_pp_accel: PP accelerations [n][3] per species (stream order)."""
        ns = len(species)
        app = [torch.empty((s.n, 3), dtype=torch.float32, device=self.device) for s in species]
        arr = _species_array(species)
        check(self.lib.pm_pp_accel(self.h, arr, ns, float(r_soft),
                                   (ctypes.c_void_p * ns)(*[_ptr(t) for t in app]),
                                   _ptr(app_max)), "pm_pp_accel")
        return app

    def step_pp(self, species, dt: float, r_soft: float, out=None, want_perm: bool = False):
        """pm_step_pp; with want_perm also the re-sort (new -> old stream position)."""
        if out is None:
            out = [self.empty_like(s) for s in species]
        a, b = _species_array(species), _species_array(out)
        perms = [torch.empty(s.n, dtype=torch.int64, device=self.device) for s in species] \
            if want_perm else None
        pp = (ctypes.c_void_p * len(species))(*[_ptr(p) for p in perms]) if perms else None
        check(self.lib.pm_step_pp(self.h, a, b, len(species), float(dt), float(r_soft), pp),
              "pm_step_pp")
        return (out, perms) if want_perm else out

    @classmethod
    def two_level(cls, n_mesh: int, n_cell: int, brick: int | None = None,
                  ratio: int = 4, r_split: float | None = None, G: float = G_UNIT,
                  soft_cells: float = 1.0, device: str = "cuda", box: float = 1.0):
        """A fine (short-range) and a coarse (long-range) context of the two-level force:
        coarse mesh n_mesh / ratio, the same softening length, r_split = 1.25 coarse cells
        unless given."""
        nc_mesh = n_mesh // ratio
        if r_split is None:
            r_split = 1.25 * box / nc_mesh
        if brick is None:
            brick = cls.default_brick(n_mesh, n_cell)
        fine = cls(n_mesh, n_cell, brick, G, soft_cells, device, box, cls.KERNEL_SHORT,
                   r_split)
        coarse = cls(nc_mesh, n_cell, brick, G, soft_cells * nc_mesh / n_mesh, device, box,
                     cls.KERNEL_LONG, r_split)
        return fine, coarse

    def interp_accel(self, species, acc: torch.Tensor, out=None, accumulate: bool = False):
        """pm_interp_accel: CIC interpolation of force meshes acc [3][n^3] to compressed
        particles, [n][3] per species (stream order)."""
        ns = len(species)
        if out is None:
            out = [torch.empty((s.n, 3), dtype=torch.float32, device=self.device)
                   for s in species]
        arr = _species_array(species)
        check(self.lib.pm_interp_accel(self.h, arr, ns, _ptr(acc.contiguous()),
                                       (ctypes.c_void_p * ns)(*[_ptr(t) for t in out]),
                                       1 if accumulate else 0), "pm_interp_accel")
        return out

    def step_p3m(self, coarse: "PMContext", species, dt: float, r_soft: float = 0.0,
                 out=None, want_perm: bool = False):
        """pm_step_p3m with this context as the fine (short-range) one."""
        if out is None:
            out = [self.empty_like(s) for s in species]
        a, b = _species_array(species), _species_array(out)
        perms = [torch.empty(s.n, dtype=torch.int64, device=self.device) for s in species] \
            if want_perm else None
        pp = (ctypes.c_void_p * len(species))(*[_ptr(p) for p in perms]) if perms else None
        check(self.lib.pm_step_p3m(self.h, coarse.h, a, b, len(species), float(dt),
                                   float(r_soft), pp), "pm_step_p3m")
        return (out, perms) if want_perm else out

    def step_vjp(self, species, dt: float, lam_x1, lam_v1):
        ns = len(species)
        lam_x0 = [torch.empty_like(t) for t in lam_x1]
        lam_v0 = [torch.empty_like(t) for t in lam_v1]
        ptrs = lambda ts: (ctypes.c_void_p * ns)(*[_ptr(t.contiguous()) for t in ts])
        lx1 = [t.contiguous() for t in lam_x1]
        lv1 = [t.contiguous() for t in lam_v1]
        arr = _species_array(species)
        check(self.lib.pm_step_vjp(self.h, arr, ns, float(dt), ptrs(lx1), ptrs(lv1),
                                   ptrs(lam_x0), ptrs(lam_v0)), "pm_step_vjp")
        return lam_x0, lam_v0

    def loss_density_vjp(self, species, rho_target: torch.Tensor):
        ns = len(species)
        lam = [torch.empty((s.n, 3), dtype=torch.float32, device=self.device) for s in species]
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        arr = _species_array(species)
        check(self.lib.pm_loss_density_vjp(self.h, arr, ns, _ptr(rho_target.contiguous()),
                                           _ptr(loss),
                                           (ctypes.c_void_p * ns)(*[_ptr(t) for t in lam])),
              "pm_loss_density_vjp")
        return loss, lam

    def reduce(self, species, rho: torch.Tensor | None = None,
               acc: torch.Tensor | None = None) -> np.ndarray:
        """pm_reduce: [mesh mass, particle mass, sum m v (3), sum m a (3), then per
        species m sum v (3), m sum a (3)] as float64."""
        out = torch.zeros(8 + 6 * len(species), dtype=torch.float64, device=self.device)
        arr = _species_array(species) if species else None
        check(self.lib.pm_reduce(self.h, arr, len(species), _ptr(rho), _ptr(acc), _ptr(out)),
              "pm_reduce")
        return out.cpu().numpy()

    def reduce_noalloc(self, species, out: torch.Tensor, rho: torch.Tensor | None = None,
                       acc: torch.Tensor | None = None) -> torch.Tensor:
        """pm_reduce_noalloc into a caller-owned float64 tensor of 8 + 6 n_sp entries
        (asynchronous; the library allocates nothing)."""
        if out.dtype != torch.float64 or out.numel() < 8 + 6 * len(species):
            raise ValueError("out must be float64 with 8 + 6 n_sp entries")
        arr = _species_array(species) if species else None
        check(self.lib.pm_reduce_noalloc(self.h, arr, len(species), _ptr(rho), _ptr(acc),
                                         _ptr(out)), "pm_reduce_noalloc")
        return out

    def pack_size(self, cs: CompressedSpecies) -> int:
        v = ctypes.c_int64()
        a = cs.c()
        check(self.lib.pm_pack_size(self.h, ctypes.byref(a), ctypes.byref(v)), "pm_pack_size")
        return v.value

    def pack(self, cs: CompressedSpecies, species_id: int = 0) -> bytes:
        size = self.pack_size(cs)
        buf = torch.empty(max(size, 64), dtype=torch.uint8, device=self.device)
        used = torch.zeros(1, dtype=torch.int64, device=self.device)
        a = cs.c()
        check(self.lib.pm_pack(self.h, ctypes.byref(a), int(species_id), _ptr(buf), size,
                               _ptr(used)), "pm_pack")
        self.sync()
        return buf[: int(used.item())].cpu().numpy().tobytes()

    def unpack(self, data: bytes, n: int, cap_esc: int | None = None):
        import struct
        w = struct.unpack("<I", data[36:40])[0] if len(data) >= 64 else 0
        w = w if w in (0x101, 0x102, 0x202) else 0  # anything else: pm_unpack rejects it
        out = self.empty_compressed(n, 0.0, cap_esc, w)
        a = out.c()
        mass = ctypes.c_double()
        sid = ctypes.c_int32()
        raw = (ctypes.c_uint8 * len(data)).from_buffer_copy(data)
        check(self.lib.pm_unpack(self.h, ctypes.cast(raw, ctypes.c_void_p), len(data),
                                 ctypes.byref(a), ctypes.byref(mass), ctypes.byref(sid)),
              "pm_unpack")
        out.mass = mass.value
        return out, sid.value

    STAGES = ["cell_offsets", "deposit", "fft_x_r2c", "fft_y_fwd", "fft_z",
              "fft_y_inv", "fft_x_c2r", "interp_kick_drift", "resort", "codec", "adjoint",
              "pp", "interp", "force_grad"]

    def profile(self, enable: bool = True):
        check(self.lib.pm_profile(self.h, 1 if enable else 0), "pm_profile")

    def profile_read(self) -> dict:
        k = len(self.STAGES)
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int64 * k)()
        check(self.lib.pm_profile_read(self.h, ms, cnt, k), "pm_profile_read")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(self.STAGES)}

    def kernel_table(self) -> torch.Tensor:
        m = self.n_mesh // 2
        t = torch.empty(3 * m * m + 1, dtype=torch.float32, device=self.device)
        check(self.lib.pm_kernel_table(self.h, _ptr(t), t.numel()), "pm_kernel_table")
        return t

    # ------------------------------------------------------- host transfers --
    def to_host(self, cs: CompressedSpecies) -> dict:
        """Compressed species -> the oracle's state dict (numpy arrays)."""
        self.sync()
        h = cs.header()
        esc = cs.esc[: h["n_esc"]].cpu().numpy().astype(np.uint64).reshape(-1, 2)
        pos = cs.pos.cpu().numpy()
        vel = cs.vel.cpu().numpy()
        st = {"n_c": self.n_cell, "brick": self.brick,
              "count": cs.count.cpu().numpy(), "esc": esc,
              "pos": pos if cs.pos_bytes == 1 else pos.view(np.uint16),
              "vel": vel.view(np.uint16) if cs.vel_bytes == 2 else vel,
              "v_max": h["v_max"], "j_min": h["j_min"], "j_max": h["j_max"]}
        if cs.widths:
            st["pos_bytes"], st["vel_bytes"] = cs.pos_bytes, cs.vel_bytes
        return st

    def from_host(self, st: dict, mass: float, cap_esc: int | None = None) -> CompressedSpecies:
        """Oracle state dict -> device compressed species (header j_min/j_max derived)."""
        import struct
        n = int(st["pos"].shape[0])
        w = widths_word(int(st.get("pos_bytes", 1)), int(st.get("vel_bytes", 2)))
        cs = self.empty_compressed(n, mass, cap_esc, w)
        cs.count.copy_(torch.from_numpy(np.ascontiguousarray(st["count"])))
        if n:
            pos = np.ascontiguousarray(st["pos"])
            vel = np.ascontiguousarray(st["vel"])
            cs.pos.copy_(torch.from_numpy(pos if cs.pos_bytes == 1 else pos.view(np.int16)))
            cs.vel.copy_(torch.from_numpy(vel.view(np.int16) if cs.vel_bytes == 2 else vel))
        esc = np.asarray(st["esc"], dtype=np.uint64).reshape(-1, 2)
        if esc.shape[0] > cs.esc.shape[0]:
            raise ValueError("escape table larger than capacity")
        if esc.shape[0]:
            cs.esc[: esc.shape[0]].copy_(torch.from_numpy(esc.view(np.int64)))
        vel = np.asarray(st["vel"])
        jmin = int(vel.min()) if n else 65536
        jmax = int(vel.max()) if n else -1
        h = struct.pack("<fiiiqq", float(st["v_max"]), jmin, jmax, 0, esc.shape[0], 0)
        cs.hdr.copy_(torch.frombuffer(bytearray(h), dtype=torch.uint8))
        return cs
