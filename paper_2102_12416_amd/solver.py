"""Python face of libjc: a context bound to a torch-allocated arena and stream.

torch provides the device memory (one uint8 arena per context) and the HIP
stream; every computation is a libjc call.  Fields cross the boundary as
device tensors holding the global padded grid ((nz+2, ny+2, nx+2) float64,
x fastest).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from ._lib import check


def _stream_handle(stream: torch.cuda.Stream) -> int:
    return int(stream.cuda_stream)


class Solver:
    """One Jacobi3D context (a decomposed grid) on one GPU.

    grid: interior (nx, ny, nz).  Either block_dims (uniform blocks; the
    last block of an axis takes the remainder) or cuts (three lists of
    block edges, a rectilinear decomposition) chooses the blocks; neither
    means one block.  mode: 'staged' (pack, exchange, unpack, sweep
    kernels) or 'fused' (one launch per iteration).  temporal: a one-block
    context advances iterate/solve windows two sweeps per launch.  overlap
    (staged mode): boundary tiles sweep first, then the halo of the new
    iterate moves on a second stream while the interior tiles sweep.
    resident: a small one-block grid (at most 32 planes, (nx + 1) / 2 * ny
    <= 512) runs each iterate/solve window as one launch that keeps the
    grid on chip."""

    def __init__(self, grid, block_dims=None, cuts=None, mode="staged", with_source=False,
                 tile_y=0, z_chunk=0, use_graphs=True, ir_dtype=None, device="cuda:0", stream=None,
                 tile_x=0, exchange="device", temporal=False, overlap=False, resident=False):
        # temporal: False, True (two sweeps per launch), or 2 / 3 sweeps per launch
        self.grid = tuple(int(v) for v in grid)
        self.device = torch.device(device)
        self.opt = L.Options()
        self.opt.mode = {"staged": L.JC_MODE_STAGED, "fused": L.JC_MODE_FUSED}[mode]
        self.opt.with_source = int(bool(with_source))
        self.opt.ir_dtype = L.JC_NONE
        if ir_dtype is not None:
            self.opt.ir_enable = 1
            self.opt.ir_dtype = {"f64": L.JC_F64, "f32": L.JC_F32, "bf16": L.JC_BF16}[ir_dtype]
        self.opt.tile_x = int(tile_x)
        self.opt.exchange = {"device": L.JC_EXCHANGE_DEVICE, "host": L.JC_EXCHANGE_HOST,
                             "metadata": L.JC_EXCHANGE_METADATA}[exchange]
        self.opt.tile_y = int(tile_y)
        self.opt.z_chunk = int(z_chunk)
        self.opt.use_graphs = int(bool(use_graphs))
        self.opt.temporal = int(bool(temporal))
        self.opt.sweeps_per_launch = 3 if temporal == 3 else 0
        self.opt.overlap = int(bool(overlap))
        self.opt.resident = int(bool(resident))
        self.with_source = bool(with_source)
        self._ctx = ctypes.c_void_p()
        g = L.i64(self.grid)
        if cuts is not None:
            arrs = [L.i64(c) for c in cuts]
            ptrs = (ctypes.POINTER(ctypes.c_int64) * 3)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_int64))
                                                          for a in arrs])
            n = L.i64([len(c) for c in cuts])
            check(L.lib.jc_create_rectilinear(g, ptrs, n, ctypes.byref(self.opt), ctypes.byref(self._ctx)))
        else:
            bd = L.i64(block_dims if block_dims is not None else self.grid)
            check(L.lib.jc_create(g, bd, ctypes.byref(self.opt), ctypes.byref(self._ctx)))
        fp = ctypes.c_size_t()
        if cuts is not None:
            check(L.lib.jc_footprint_rectilinear(g, ptrs, n, ctypes.byref(self.opt), ctypes.byref(fp)))
        else:
            check(L.lib.jc_footprint(g, bd, ctypes.byref(self.opt), ctypes.byref(fp)))
        self.footprint = int(fp.value)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.arena = torch.empty(self.footprint + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        self._arena_off = (-base) % 256
        self.arena.record_stream(self.stream)
        check(L.lib.jc_bind(self._ctx, ctypes.c_void_p(base + self._arena_off), self.footprint,
                            ctypes.c_void_p(_stream_handle(self.stream))))

    # ------------------------------------------------------------ lifetime
    def close(self):
        if self._ctx:
            L.lib.jc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------- fields
    def padded_shape(self):
        nx, ny, nz = self.grid
        return (nz + 2, ny + 2, nx + 2)

    def _device_field(self, a):
        t = torch.as_tensor(a)
        if t.dtype != torch.float64 or tuple(t.shape) != self.padded_shape():
            raise ValueError("field must be float64 of shape %s" % (self.padded_shape(),))
        t = t.to(self.device).contiguous()
        return t

    def load(self, u0, b=None):
        """Load the initial iterate (shell = Dirichlet values) and the source."""
        cur = torch.cuda.current_stream(self.device)
        tu = self._device_field(u0)
        tb = self._device_field(b) if b is not None else None
        self.stream.wait_stream(cur)
        check(L.lib.jc_load_field(self._ctx, L.JC_FIELD_U, ctypes.c_void_p(tu.data_ptr())))
        tu.record_stream(self.stream)
        if tb is not None:
            check(L.lib.jc_load_field(self._ctx, L.JC_FIELD_B, ctypes.c_void_p(tb.data_ptr())))
            tb.record_stream(self.stream)
        return self

    def store(self, which=L.JC_FIELD_U) -> torch.Tensor:
        """Current iterate (or the source) as a global padded device tensor."""
        out = torch.zeros(self.padded_shape(), dtype=torch.float64, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        check(L.lib.jc_store_field(self._ctx, which, ctypes.c_void_p(out.data_ptr())))
        out.record_stream(self.stream)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    # ------------------------------------------------------------ hot path
    def pack_faces(self):
        check(L.lib.jc_pack_faces(self._ctx))

    def exchange(self):
        check(L.lib.jc_exchange(self._ctx))

    def unpack_faces(self):
        check(L.lib.jc_unpack_faces(self._ctx))

    def sweep(self):
        check(L.lib.jc_sweep(self._ctx))

    def iterate(self, n: int):
        check(L.lib.jc_iterate(self._ctx, int(n)))

    def residual(self) -> float:
        r = ctypes.c_double()
        check(L.lib.jc_residual(self._ctx, ctypes.byref(r)))
        return r.value

    def solve(self, rtol=0.0, max_iter=1000, check_every=10, history=False):
        """Returns a dict with iters, rel_resid, abs_resid, r0, status, history."""
        info = L.SolveInfo()
        buf = None
        if history:
            cap = max_iter // max(check_every, 1) + 3
            buf = (ctypes.c_double * cap)()
            info.history = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
            info.history_cap = cap
        st = check(L.lib.jc_solve(self._ctx, float(rtol), int(max_iter), int(check_every), ctypes.byref(info)))
        out = dict(iters=info.iters, checks=info.outer, rel_resid=info.rel_resid, abs_resid=info.abs_resid,
                   r0=info.r0, status=st, converged=(st == L.JC_OK))
        if buf is not None:
            out["history"] = [buf[i] for i in range(info.history_len)]
        return out

    def solve_ir(self, inner=50, rtol=1e-10, max_inner=20000, history=False):
        """Mixed-precision iterative refinement (needs ir_dtype at creation).
        Returns a dict like solve(); iters counts inner sweeps, outer the
        residual checks."""
        info = L.SolveInfo()
        buf = None
        if history:
            cap = max_inner // max(inner, 1) + 3
            buf = (ctypes.c_double * cap)()
            info.history = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
            info.history_cap = cap
        st = check(L.lib.jc_solve_ir(self._ctx, int(inner), float(rtol), int(max_inner), ctypes.byref(info)))
        out = dict(iters=info.iters, outer=info.outer, rel_resid=info.rel_resid, abs_resid=info.abs_resid,
                   r0=info.r0, status=st, converged=(st == L.JC_OK))
        if buf is not None:
            out["history"] = [buf[i] for i in range(info.history_len)]
        return out

    def synchronize(self):
        self.stream.synchronize()

    # -------------------------------------------------------- introspection
    @property
    def num_blocks(self):
        return int(L.lib.jc_num_blocks(self._ctx))

    @property
    def num_pairs(self):
        return int(L.lib.jc_num_pairs(self._ctx))

    @property
    def iterations(self):
        return int(L.lib.jc_iterations(self._ctx))

    def block_info(self, i):
        out = (ctypes.c_int64 * 17)()
        check(L.lib.jc_block_info(self._ctx, int(i), out))
        v = list(out)
        return dict(n=tuple(v[0:3]), off=tuple(v[3:6]), nbr=tuple(v[6:12]), pitch=v[12], plane=v[13],
                    u_off=(v[14], v[15]), parity=v[16])

    def pair_info(self, i):
        out = (ctypes.c_int64 * 10)()
        check(L.lib.jc_pair_info(self._ctx, int(i), out))
        v = list(out)
        return dict(src_block=v[0], src_face=v[1], dst_block=v[2], dst_face=v[3], count=v[4], slow=v[5],
                    fast=v[6], buf_off=v[7], recv_off=v[8], ld=v[9])

    def face_buffer(self, q, slot):
        """Values of pair q's send (slot 0) or receive (slot 1) buffer, (slow, fast)."""
        p = self.pair_info(q)
        flat = self.arena_view(p["buf_off"] if slot == 0 else p["recv_off"], p["slow"] * p["ld"])
        return flat.view(p["slow"], p["ld"])[:, :p["fast"]]

    def tile_info(self):
        out = (ctypes.c_int64 * 4)()
        check(L.lib.jc_tile_info(self._ctx, out))
        return dict(tile_x=out[0], tile_y=out[1], z_chunk=out[2], items=out[3])

    def set_temporal_tiles(self, rows, z_chunk):
        check(L.lib.jc_set_temporal_tiles(self._ctx, int(rows), int(z_chunk)))

    def temporal_info(self):
        out = (ctypes.c_int64 * 3)()
        check(L.lib.jc_temporal_info(self._ctx, out))
        return dict(temporal=bool(out[0]), sweeps=int(out[0]), rows=out[1], z_chunk=out[2])

    def arena_view(self, byte_off, count, dtype=torch.float64):
        """A tensor view of `count` elements of the arena at `byte_off` (tests)."""
        esz = torch.empty((), dtype=dtype).element_size()
        start = self._arena_off + int(byte_off)
        return self.arena[start:start + count * esz].view(dtype)

    def block_array(self, i, copy=None):
        """The padded array of block i (copy = current if None) as a 3D view
        (nz+2, ny+2, pitch) starting at element (0,0,0)."""
        info = self.block_info(i)
        nx, ny, nz = info["n"]
        c = info["parity"] if copy is None else copy
        flat = self.arena_view(info["u_off"][c], info["plane"] * (nz + 2))
        return flat.view(nz + 2, ny + 2, info["pitch"])

    def set_tiles(self, tile_x, tile_y, z_chunk):
        check(L.lib.jc_set_tiles(self._ctx, int(tile_x), int(tile_y), int(z_chunk)))

    def autotune(self, reps=5):
        """Pick the fastest tile shape for this context (and, with temporal
        blocking, the fastest two-sweep shape: temporal_info()); returns
        (tile_x, tile_y, z_chunk, microseconds per sweep)."""
        out = (ctypes.c_int64 * 4)()
        check(L.lib.jc_autotune(self._ctx, int(reps), out))
        return tuple(out)

    # -------------------------------------------------------------- timing
    def set_pace(self, ticks):
        """Pace of the solve-loop sweep (jc_set_pace): ticks of the GPU's
        100 MHz clock per plane step; 0 = none."""
        check(L.lib.jc_set_pace(self._ctx, int(ticks)))

    @property
    def pace(self):
        return int(L.lib.jc_get_pace(self._ctx))

    def autotune_pace(self, reps=10):
        """Tune the pace for the current tile shape (jc_autotune_pace);
        returns (pace, us per sweep with it, us per sweep without)."""
        out = (ctypes.c_int64 * 3)()
        check(L.lib.jc_autotune_pace(self._ctx, int(reps), out))
        return tuple(int(v) for v in out)

    def set_timing(self, enable=True):
        check(L.lib.jc_set_timing(self._ctx, int(bool(enable))))

    def kernel_time(self, kind):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(L.lib.jc_kernel_time(self._ctx, int(kind), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def min_surface_parts(grid, nblocks):
    out = (ctypes.c_int64 * 3)()
    check(L.lib.jc_min_surface_parts(L.i64(grid), int(nblocks), out))
    return tuple(out)


def footprint(grid, block_dims=None, with_source=False, mode="staged"):
    opt = L.Options()
    opt.mode = {"staged": L.JC_MODE_STAGED, "fused": L.JC_MODE_FUSED}[mode]
    opt.with_source = int(bool(with_source))
    opt.ir_dtype = L.JC_NONE
    fp = ctypes.c_size_t()
    bd = block_dims if block_dims is not None else grid
    check(L.lib.jc_footprint(L.i64(grid), L.i64(bd), ctypes.byref(opt), ctypes.byref(fp)))
    return int(fp.value)


class Group:
    """Several bound, loaded Solvers swept by shared launches (libjc group).

    The members must not be used on their own streams while the group
    exists; close() (or leaving a with-block) releases it.
    static_scratch: bind to the library's static device scratch
    (jc_group_bind_static, no allocation; one such group per device at a
    time) instead of a torch-allocated buffer."""

    def __init__(self, solvers, use_graphs=True, stream=None, tile=None, temporal=False, static_scratch=False,
                 resident=False):
        # temporal: False, True (two sweeps of every member per launch) or 3;
        # resident: every window one launch, one work-group per member
        self.solvers = list(solvers)
        dev = self.solvers[0].device
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s._ctx.value for s in self.solvers])
        self._g = ctypes.c_void_p()
        tl = None if tile is None else (ctypes.c_int * 3)(*[int(v) for v in tile])
        flags = (1 if use_graphs else 0) | (4 if temporal == 3 else 2 if temporal else 0) | (8 if resident else 0)
        check(L.lib.jc_group_create(arr, len(self.solvers), ctypes.c_void_p(_stream_handle(self.stream)),
                                    flags, tl, ctypes.byref(self._g)))
        fp = ctypes.c_size_t()
        check(L.lib.jc_group_footprint(self._g, ctypes.byref(fp)))
        self.footprint = int(fp.value)
        if static_scratch:
            self.scratch = None
            try:
                check(L.lib.jc_group_bind_static(self._g))
            except Exception:
                self.close()
                raise
            return
        self.scratch = torch.empty(int(fp.value) + 256, dtype=torch.uint8, device=dev)
        base = self.scratch.data_ptr()
        off = (-base) % 256
        self.scratch.record_stream(self.stream)
        check(L.lib.jc_group_bind(self._g, ctypes.c_void_p(base + off), int(fp.value)))

    def iterate(self, n):
        check(L.lib.jc_group_iterate(self._g, int(n)))

    def residuals(self):
        out = (ctypes.c_double * len(self.solvers))()
        check(L.lib.jc_group_residuals(self._g, out))
        return list(out)

    def check(self, rtol, max_iter):
        """The stopping rule of every member (jc_group_check): a list of
        (relative residual, done) pairs."""
        rel = (ctypes.c_double * len(self.solvers))()
        done = (ctypes.c_int * len(self.solvers))()
        check(L.lib.jc_group_check(self._g, float(rtol), int(max_iter), rel, done))
        return [(rel[i], bool(done[i])) for i in range(len(self.solvers))]

    def close(self):
        if self._g:
            L.lib.jc_group_destroy(self._g)
            self._g = ctypes.c_void_p()
            for s in self.solvers:
                s.stream.wait_stream(self.stream)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def synth_field(grid, seed, kind, device="cuda:0", stream=None):
    """Device tensor (nz+2, ny+2, nx+2) float64 with the seeded synthetic
    boundary field (kind 0) or source (kind 1), generated on the GPU."""
    nx, ny, nz = (int(v) for v in grid)
    dev = torch.device(device)
    out = torch.empty((nz + 2, ny + 2, nx + 2), dtype=torch.float64, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    check(L.lib.jc_synth_field(ctypes.c_void_p(out.data_ptr()), L.i64((nx, ny, nz)), int(seed) & ((1 << 64) - 1),
                               int(kind), ctypes.c_void_p(_stream_handle(st))))
    return out
