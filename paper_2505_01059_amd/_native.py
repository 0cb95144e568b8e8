"""ctypes binding of libmtp.so (argument marshalling only).

Every entry point of include/mtp.h appears here under the same name.  Device
memory comes from torch (one uint8 workspace tensor per object) and work is
enqueued on torch's current stream of that device.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, byref, c_char_p, c_float, c_int32, c_size_t, c_uint32, c_uint64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(HERE, "libmtp.so")


class MtpError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"mtp status {status}: {msg}")


STAGE_CANDIDATES, STAGE_ROLLOUT, STAGE_TOPK, STAGE_UPDATE, STAGE_ALL = range(5)
MTP_ABI_VERSION = 3


class mtp_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", c_uint32), ("dynamics", c_int32), ("interp", c_int32), ("n_links", c_int32),
        ("state_dim", c_int32), ("ctrl_dim", c_int32), ("horizon", c_int32), ("n_layers", c_int32),
        ("n_width", c_int32), ("n_tensor", c_int32), ("n_gauss", c_int32), ("n_elites", c_int32),
        ("n_iters", c_int32), ("bspline_degree", c_int32),
        ("temperature", c_float), ("smoothing", c_float), ("sigma_min", c_float), ("sigma_init", c_float),
        ("u_min", c_float), ("u_max", c_float), ("dt", c_float),
        ("seed", c_uint64),
        ("task_params", POINTER(c_float)), ("n_task_params", c_int32),
        ("sample_params", POINTER(c_float)), ("n_debug_states", c_int32),
        ("n_replicas", c_int32), ("sample_wor", c_int32), ("diagnostics", c_int32),
    ]


class mtp_buffers(ctypes.Structure):
    _fields_ = [(name, c_void_p) for name in
                ("Z", "I", "U", "cost", "elite_idx", "elite_cost", "weights", "mu", "sigma", "x0",
                 "action", "X_dbg", "entropy")] + [("ld_U", c_size_t)]


_LIB = None


def load():
    """Load libmtp.so; raises if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2505_01059_amd.build`")
    # torch first: its HIP runtime then satisfies the library's libamdhip64.so.7.
    # Loaded the other way round, torch (which asks for libamdhip64.so by file
    # name) maps a second runtime, and its streams are foreign to the library's.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "mtp_workspace_bytes": (c_size_t, [P]),
        "mtp_transient_bytes": (c_size_t, [P]),
        "mtp_resident_bytes": (c_size_t, [P]),
        "mtp_validate_config": (c_int32, [P, c_char_p, c_size_t]),
        "mtp_plan_create": (c_int32, [P, P, c_size_t, P, POINTER(P)]),
        "mtp_replan": (c_int32, [P, P, c_int32]),
        "mtp_replan_at": (c_int32, [P, P, c_int32, c_uint32]),
        "mtp_get_action": (c_int32, [P, P]),
        "mtp_get_state": (c_int32, [P, P, P, POINTER(c_uint32)]),
        "mtp_set_state": (c_int32, [P, P, P, c_uint32]),
        "mtp_run_stage": (c_int32, [P, c_int32, c_uint32, c_int32]),
        "mtp_set_x0": (c_int32, [P, P]),
        "mtp_set_graph_mode": (c_int32, [P, c_int32]),
        "mtp_plan_draws_ahead": (c_int32, [P]),
        "mtp_get_buffers": (c_int32, [P, P]),
        "mtp_get_flags": (c_int32, [P, POINTER(c_uint32)]),
        "mtp_plan_destroy": (c_int32, [P]),
        "mtp_status_str": (c_char_p, [c_int32]),
        "mtp_last_error": (c_char_p, [P]),
        "mtp_supported_chain_links": (c_int32, [POINTER(c_int32), c_int32]),
        "mtp_interp_table": (c_int32, [P, P, P]),
        "mtp_set_stage_timing": (c_int32, [P, c_int32]),
        "mtp_batch_workspace_bytes": (c_size_t, [P, c_int32]),
        "mtp_batch_create": (c_int32, [P, c_int32, P, c_size_t, P, POINTER(P)]),
        "mtp_batch_replan": (c_int32, [P, P, P]),
        "mtp_batch_step": (c_int32, [P, c_int32, P, P, P, P, P, P]),
        "mtp_batch_get_actions": (c_int32, [P, P]),
        "mtp_batch_get_buffers": (c_int32, [P, c_int32, P]),
        "mtp_batch_set_state": (c_int32, [P, c_int32, P, P]),
        "mtp_batch_set_schedule": (c_int32, [P, c_int32, c_int32]),
        "mtp_batch_autotune": (c_int32, [P, c_int32, P, P]),
        "mtp_batch_set_schedule_full": (c_int32, [P, P]),
        "mtp_batch_get_schedule": (c_int32, [P, P]),
        "mtp_batch_tune": (c_int32, [P, c_int32, c_char_p, P, POINTER(c_float), POINTER(c_int32)]),
        "mtp_batch_mix_signature": (c_uint64, [P, c_int32]),
        "mtp_schedule_cache_lookup": (c_int32, [c_char_p, c_char_p, c_int32, c_uint64, P, POINTER(c_float),
                                                POINTER(c_int32)]),
        "mtp_schedule_cache_store": (c_int32, [c_char_p, c_char_p, c_int32, c_uint64, P, c_float]),
        "mtp_batch_set_graph_mode": (c_int32, [P, c_int32]),
        "mtp_batch_destroy": (c_int32, [P]),
        "mtp_batch_last_error": (c_char_p, [P]),
        "mtp_server_workspace_bytes": (c_size_t, [c_size_t, c_int32, c_uint32]),
        "mtp_server_create": (c_int32, [c_size_t, c_int32, c_uint32, c_int32, c_int32, P, c_size_t, P,
                                        POINTER(P)]),
        "mtp_server_create_simulated": (c_int32, [c_size_t, c_int32, c_uint32, c_int32, c_int32, ctypes.c_double,
                                                  POINTER(P)]),
        "mtp_server_add_robot": (c_int32, [P, P, POINTER(c_int32)]),
        "mtp_server_remove_robot": (c_int32, [P, c_int32]),
        "mtp_server_get_robot_state": (c_int32, [P, c_int32, P, P, POINTER(c_uint32)]),
        "mtp_server_submit": (c_int32, [P, c_int32, P, c_int32, c_uint64, POINTER(c_uint64)]),
        "mtp_server_pump": (c_int32, [P, c_int32, POINTER(c_int32)]),
        "mtp_server_poll": (c_int32, [P, P, c_int32, POINTER(c_int32)]),
        "mtp_server_get_stats": (c_int32, [P, P]),
        "mtp_server_now_ns": (c_uint64, []),
        "mtp_server_destroy": (c_int32, [P]),
        "mtp_server_last_error": (c_char_p, [P]),
        "mtp_get_stage_times": (c_int32, [P, P, P]),
        "mtp_plant_step": (c_int32, [P, P, P, P]),
        "mtp_noalloc_scratch_bytes": (c_size_t, []),
        "mtp_replan_noalloc": (c_int32, [P, P, P, P, c_int32, c_uint32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


# ------------------------------------------------------------------ marshalling

def task_params_of(cfg) -> np.ndarray:
    """Flatten a workload's task into the float32 layout documented in mtp.h."""
    t = cfg.task
    if cfg.dynamics == 0:
        obs = np.asarray(t.obstacles, np.float32).reshape(-1, 3)
        head = np.array([t.goal[0], t.goal[1], t.goal_weight, t.obstacle_penalty, t.ctrl_weight,
                         obs.shape[0]], np.float32)
        return np.concatenate([head, obs.ravel()]).astype(np.float32)
    head = np.array([t.gravity, t.goal_weight, t.ctrl_weight, t.target[0], t.target[1]], np.float32)
    parts = [head, np.asarray(t.masses, np.float32), np.asarray(t.lengths, np.float32)]
    if cfg.dynamics == 2:
        parts.append(np.array([t.ground_y, t.k_contact, t.d_contact, t.v_slip], np.float32))
    return np.concatenate(parts).astype(np.float32)


def config_struct(cfg, n_debug_states=0):
    """Build an mtp_config; returns (struct, keepalive arrays)."""
    task = np.ascontiguousarray(task_params_of(cfg), dtype=np.float32)
    keep = [task]
    c = mtp_config()
    c.abi_version = MTP_ABI_VERSION
    c.dynamics = int(cfg.dynamics)
    c.interp = int(cfg.interp)
    c.n_links = int(cfg.n_links)
    c.state_dim = int(cfg.state_dim)
    c.ctrl_dim = int(cfg.ctrl_dim)
    c.horizon = int(cfg.horizon)
    c.n_layers = int(cfg.n_layers)
    c.n_width = int(cfg.n_width)
    c.n_tensor = int(cfg.n_tensor)
    c.n_gauss = int(cfg.n_gauss)
    c.n_elites = int(cfg.n_elites)
    c.n_iters = int(cfg.n_iters)
    c.bspline_degree = int(cfg.bspline_degree)
    c.temperature = float(cfg.temperature)
    c.smoothing = float(cfg.smoothing)
    c.sigma_min = float(cfg.sigma_min)
    c.sigma_init = float(cfg.sigma_init)
    c.u_min = float(cfg.u_min)
    c.u_max = float(cfg.u_max)
    c.dt = float(cfg.dt)
    c.seed = int(cfg.seed) & 0xFFFFFFFFFFFFFFFF
    c.task_params = task.ctypes.data_as(POINTER(c_float))
    c.n_task_params = int(task.size)
    if cfg.sample_params is not None:
        sp = np.ascontiguousarray(cfg.sample_params, dtype=np.float32)
        keep.append(sp)
        c.sample_params = sp.ctypes.data_as(POINTER(c_float))
    c.n_debug_states = int(n_debug_states)
    c.n_replicas = int(getattr(cfg, "n_replicas", 1))
    c.sample_wor = int(getattr(cfg, "sample_wor", 0))
    c.diagnostics = int(getattr(cfg, "diagnostics", 0))
    return c, keep


def _check(lib, status, obj=None):
    if status != 0:
        msg = lib.mtp_status_str(status).decode()
        if obj:
            msg += ": " + lib.mtp_last_error(obj).decode()
        raise MtpError(status, msg)


def validate(cfg, n_debug_states=0):
    """(status, reason) of the library's config check; touches no device."""
    lib = load()
    c, keep = config_struct(cfg, n_debug_states)
    buf = ctypes.create_string_buffer(256)
    st = lib.mtp_validate_config(byref(c), buf, 256)
    return st, buf.value.decode()


def interp_table(cfg):
    """(basis (T, 8) float32, span (T,) int32) as the library builds them on the host."""
    lib = load()
    c, keep = config_struct(cfg)
    basis = np.zeros((cfg.horizon, 8), np.float32)
    span = np.zeros(cfg.horizon, np.int32)
    _check(lib, lib.mtp_interp_table(byref(c), basis.ctypes.data_as(c_void_p), span.ctypes.data_as(c_void_p)))
    return basis, span


def workspace_bytes(cfg, n_debug_states=0):
    lib = load()
    c, keep = config_struct(cfg, n_debug_states)
    return int(lib.mtp_workspace_bytes(byref(c)))


def transient_bytes(cfg) -> int:
    """Bytes one replan of cfg borrows from a server's pool (0 if invalid)."""
    c, keep = config_struct(cfg)
    return int(load().mtp_transient_bytes(byref(c)))


def resident_bytes(cfg) -> int:
    """Bytes a server keeps in its pool while the robot of cfg is registered (0 if invalid)."""
    c, keep = config_struct(cfg)
    return int(load().mtp_resident_bytes(byref(c)))


def plant_step(cfg, x, u):
    """One float64 host step of cfg's model from state x under control u (the
    robot that executes the planner's action)."""
    c, keep = config_struct(cfg)
    xx = np.ascontiguousarray(np.asarray(x, np.float64))
    uu = np.ascontiguousarray(np.asarray(u, np.float32))
    out = np.empty_like(xx)
    _check(load(), load().mtp_plant_step(byref(c), xx.ctypes.data_as(c_void_p), uu.ctypes.data_as(c_void_p),
                                         out.ctypes.data_as(c_void_p)))
    return out


def _torch():
    import torch
    return torch


class Plan:
    """One planner instance (mtp_plan) with a torch-allocated workspace."""

    def __init__(self, cfg, device="cuda", n_debug_states=0, use_graph=True, workspace=None):
        torch = _torch()
        self.lib = load()
        self.cfg = cfg
        self.device = torch.device(device)
        self._c, self._keep = config_struct(cfg, n_debug_states)
        nbytes = int(self.lib.mtp_workspace_bytes(byref(self._c)))
        if nbytes == 0:
            st, why = validate(cfg, n_debug_states)
            raise MtpError(st, why)
        self.ws_bytes = nbytes
        self.workspace = workspace if workspace is not None else torch.empty(
            nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = c_void_p()
        st = self.lib.mtp_plan_create(byref(self._c), c_void_p(self.workspace.data_ptr()), nbytes,
                                      c_void_p(self.stream.cuda_stream), byref(h))
        _check(self.lib, st)
        self.handle = h
        self._x0 = None
        if not use_graph:
            self.set_graph_mode(False)

    # -- lifecycle
    def close(self):
        if getattr(self, "handle", None):
            self.lib.mtp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls
    def _x0_dev(self, x0):
        torch = _torch()
        x = torch.as_tensor(np.asarray(x0, np.float32) if not isinstance(x0, torch.Tensor) else x0,
                            dtype=torch.float32, device=self.device).contiguous()
        self._x0 = x          # keep alive until the stream has read it
        return x

    def replan(self, x0, shift=1, replan_idx=None):
        x = self._x0_dev(x0)
        if replan_idx is None:
            st = self.lib.mtp_replan(self.handle, c_void_p(x.data_ptr()), int(shift))
        else:
            st = self.lib.mtp_replan_at(self.handle, c_void_p(x.data_ptr()), int(shift), int(replan_idx))
        _check(self.lib, st, self.handle)

    def action(self):
        out = np.zeros(self.cfg.ctrl_dim, np.float32)
        _check(self.lib, self.lib.mtp_get_action(self.handle, out.ctypes.data_as(c_void_p)), self.handle)
        return out

    def get_state(self):
        torch = _torch()
        T, n = self.cfg.horizon, self.cfg.ctrl_dim
        mu = torch.empty((T, n), dtype=torch.float32, device=self.device)
        sg = torch.empty((T, n), dtype=torch.float32, device=self.device)
        r = c_uint32()
        _check(self.lib, self.lib.mtp_get_state(self.handle, c_void_p(mu.data_ptr()), c_void_p(sg.data_ptr()),
                                                byref(r)), self.handle)
        return mu, sg, int(r.value)

    def set_state(self, mu, sigma, replan_idx):
        torch = _torch()
        mu = torch.as_tensor(mu, dtype=torch.float32, device=self.device).contiguous()
        sg = torch.as_tensor(sigma, dtype=torch.float32, device=self.device).contiguous()
        self._state_keep = (mu, sg)
        _check(self.lib, self.lib.mtp_set_state(self.handle, c_void_p(mu.data_ptr()), c_void_p(sg.data_ptr()),
                                                int(replan_idx)), self.handle)

    def set_x0(self, x0):
        x = self._x0_dev(x0)
        _check(self.lib, self.lib.mtp_set_x0(self.handle, c_void_p(x.data_ptr())), self.handle)

    def run_stage(self, stage, replan_idx, k):
        _check(self.lib, self.lib.mtp_run_stage(self.handle, int(stage), int(replan_idx), int(k)), self.handle)

    def draws_ahead(self):
        """Whether each rollout also draws the next iteration's tensor-path controls."""
        return bool(self.lib.mtp_plan_draws_ahead(self.handle))

    def set_graph_mode(self, on):
        _check(self.lib, self.lib.mtp_set_graph_mode(self.handle, 1 if on else 0), self.handle)

    def set_stage_timing(self, on):
        _check(self.lib, self.lib.mtp_set_stage_timing(self.handle, 1 if on else 0), self.handle)

    def stage_times(self):
        """{stage: (total_ms, launches)} for candidates, rollout, topk, update."""
        ms = np.zeros(4, np.float64)
        cnt = np.zeros(4, np.uint64)
        _check(self.lib, self.lib.mtp_get_stage_times(self.handle, ms.ctypes.data_as(c_void_p),
                                                      cnt.ctypes.data_as(c_void_p)), self.handle)
        names = ("candidates", "rollout", "topk", "update")
        return {nm: (float(ms[i]), int(cnt[i])) for i, nm in enumerate(names)}

    def flags(self):
        f = c_uint32()
        _check(self.lib, self.lib.mtp_get_flags(self.handle, byref(f)), self.handle)
        return int(f.value)

    def buffers(self):
        """Torch views of the plan's device buffers (see mtp_buffers in mtp.h)."""
        b = mtp_buffers()
        _check(self.lib, self.lib.mtp_get_buffers(self.handle, byref(b)), self.handle)
        return _buffer_views(b, self.cfg, self.workspace, int(self._c.n_debug_states))


def _buffer_views(b, cfg, workspace, n_debug):
    torch = _torch()
    base = workspace.data_ptr()
    T, n, d = cfg.horizon, cfg.ctrl_dim, cfg.state_dim
    B, E, L, W, P = cfg.n_samples, cfg.n_elites, cfg.n_layers, cfg.n_width, cfg.n_tensor
    ld = int(b.ld_U)

    def view(ptr, dtype, shape):
        if not ptr:
            return None
        esz = torch.empty((), dtype=dtype).element_size()
        count = int(np.prod(shape))
        off = int(ptr) - base
        return workspace[off:off + count * esz].view(dtype).view(*shape)

    out = dict(
        Z=view(b.Z, torch.float32, (L, W, n)),
        I=view(b.I, torch.uint8, (L, max(P, 1)))[:, :P],
        U=view(b.U, torch.float32, (T, n, ld))[:, :, :B],
        cost=view(b.cost, torch.float32, (B,)),
        elite_idx=view(b.elite_idx, torch.int32, (E,)),
        elite_cost=view(b.elite_cost, torch.float32, (E,)),
        weights=view(b.weights, torch.float32, (E,)),
        mu=view(b.mu, torch.float32, (T, n)),
        sigma=view(b.sigma, torch.float32, (T, n)),
        x0=view(b.x0, torch.float32, (d,)),
        action=view(b.action, torch.float32, (n,)),
        entropy=view(b.entropy, torch.float32, (cfg.n_iters,)),
    )
    R = max(1, int(getattr(cfg, "n_replicas", 1)))
    out["X_all"] = view(b.X_dbg, torch.float32, (R, T, d, n_debug)) if n_debug > 0 else None
    out["X"] = out["X_all"][0] if n_debug > 0 else None
    out["ld_U"] = ld
    return out


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class mtp_batch_schedule(ctypes.Structure):
    _fields_ = [(name, c_int32) for name in
                ("wg_per_cu", "order", "cand_tiles", "roll_tiles", "refit_outputs", "split_pct")]


SCHEDULE_FIELDS = tuple(name for name, _ in mtp_batch_schedule._fields_)


def _schedule_dict(s):
    return {name: int(getattr(s, name)) for name in SCHEDULE_FIELDS}


def _schedule_struct(d):
    return mtp_batch_schedule(*[int(d[name]) for name in SCHEDULE_FIELDS])


def mix_signature(cfgs):
    """mtp_batch_mix_signature of a list of workload configs (host only)."""
    lib = load()
    structs = [config_struct(c) for c in cfgs]
    arr = (mtp_config * len(structs))(*[c for c, _ in structs])
    return int(lib.mtp_batch_mix_signature(arr, len(structs)))


def schedule_cache_lookup(path, arch, cus, mix):
    """(schedule dict, ms) stored under (arch, cus, mix) in the cache file, or None."""
    lib = load()
    out, ms, found = mtp_batch_schedule(), c_float(), c_int32()
    _check(lib, lib.mtp_schedule_cache_lookup(os.fsencode(path), arch.encode(), int(cus), int(mix), byref(out),
                                              byref(ms), byref(found)))
    return (_schedule_dict(out), float(ms.value)) if found.value else None


def schedule_cache_store(path, arch, cus, mix, schedule, ms):
    lib = load()
    s = _schedule_struct(schedule)
    _check(lib, lib.mtp_schedule_cache_store(os.fsencode(path), arch.encode(), int(cus), int(mix), byref(s),
                                             float(ms)))


class Batch:
    """Many instances replanned by one persistent launch (mtp_batch)."""

    def __init__(self, cfgs, device="cuda", use_graph=True, n_debug_states=None):
        torch = _torch()
        self.lib = load()
        self.cfgs = list(cfgs)
        self.n = len(self.cfgs)
        self.device = torch.device(device)
        self.n_debug = [0] * self.n if n_debug_states is None else [int(v) for v in n_debug_states]
        structs = [config_struct(c, nd) for c, nd in zip(self.cfgs, self.n_debug)]
        self._keep = [k for _, k in structs]
        arr = (mtp_config * self.n)(*[c for c, _ in structs])
        self._arr = arr
        nbytes = int(self.lib.mtp_batch_workspace_bytes(arr, self.n))
        if nbytes == 0:
            for i, c in enumerate(self.cfgs):
                st, why = validate(c)
                if st != 0:
                    raise MtpError(st, f"config {i}: {why}")
            raise MtpError(1, "batch layout failed")
        self.ws_bytes = nbytes
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = c_void_p()
        st = self.lib.mtp_batch_create(arr, self.n, c_void_p(self.workspace.data_ptr()), nbytes,
                                       c_void_p(self.stream.cuda_stream), byref(h))
        _check(self.lib, st)
        self.handle = h
        self.x0_sizes = [c.state_dim for c in self.cfgs]
        self.act_sizes = [c.ctrl_dim for c in self.cfgs]
        self._x0 = None
        if not use_graph:
            self.lib.mtp_batch_set_graph_mode(self.handle, 0)

    def _err(self, st):
        if st != 0:
            raise MtpError(st, self.lib.mtp_status_str(st).decode() + ": " +
                           self.lib.mtp_batch_last_error(self.handle).decode())

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mtp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack_x0(self, x0s):
        torch = _torch()
        flat = np.concatenate([np.asarray(x, np.float32).ravel() for x in x0s]).astype(np.float32)
        return torch.tensor(flat, device=self.device)

    def replan(self, x0_packed, shift=None):
        x = x0_packed
        self._x0 = x
        sh = None if shift is None else _i32(np.broadcast_to(np.asarray(shift), (self.n,)))
        self._sh = sh
        self._err(self.lib.mtp_batch_replan(self.handle, c_void_p(x.data_ptr()),
                                            None if sh is None else sh.ctypes.data_as(c_void_p)))

    def step(self, active, k_begin, k_end, shift, replan_idx, x0_packed=None):
        active, kb, ke, sh = _i32(active), _i32(k_begin), _i32(k_end), _i32(shift)
        rr = np.ascontiguousarray(np.asarray(replan_idx, dtype=np.uint32))
        self._hold = (active, kb, ke, sh, rr, x0_packed)
        self._err(self.lib.mtp_batch_step(
            self.handle, len(active), active.ctypes.data_as(c_void_p), kb.ctypes.data_as(c_void_p),
            ke.ctypes.data_as(c_void_p), sh.ctypes.data_as(c_void_p), rr.ctypes.data_as(c_void_p),
            None if x0_packed is None else c_void_p(x0_packed.data_ptr())))

    def actions(self):
        out = np.zeros(sum(self.act_sizes), np.float32)
        self._err(self.lib.mtp_batch_get_actions(self.handle, out.ctypes.data_as(c_void_p)))
        return np.split(out, np.cumsum(self.act_sizes)[:-1])

    def buffers(self, i):
        b = mtp_buffers()
        self._err(self.lib.mtp_batch_get_buffers(self.handle, int(i), byref(b)))
        return _buffer_views(b, self.cfgs[i], self.workspace, self.n_debug[i])

    def set_state(self, i, mu, sigma):
        torch = _torch()
        mu = torch.as_tensor(mu, dtype=torch.float32, device=self.device).contiguous()
        sg = torch.as_tensor(sigma, dtype=torch.float32, device=self.device).contiguous()
        self._state_keep = (mu, sg)
        self._err(self.lib.mtp_batch_set_state(self.handle, int(i), c_void_p(mu.data_ptr()),
                                               c_void_p(sg.data_ptr())))

    def schedule(self):
        s = mtp_batch_schedule()
        self._err(self.lib.mtp_batch_get_schedule(self.handle, byref(s)))
        return _schedule_dict(s)

    def set_schedule(self, wg_per_cu=None, order=None, **knobs):
        """Set any of the schedule knobs of mtp.h (the others keep their values)."""
        d = self.schedule()
        knobs.update({k: v for k, v in (("wg_per_cu", wg_per_cu), ("order", order)) if v is not None})
        unknown = set(knobs) - set(SCHEDULE_FIELDS)
        if unknown:
            raise ValueError(f"unknown schedule knobs {sorted(unknown)}")
        d.update(knobs)
        s = _schedule_struct(d)
        self._err(self.lib.mtp_batch_set_schedule_full(self.handle, byref(s)))

    def tune(self, reps=2, cache_path=None):
        """Search the schedule (or take it from the cache file); returns (schedule, ms, from_cache)."""
        out, ms, hit = mtp_batch_schedule(), c_float(), c_int32()
        self._err(self.lib.mtp_batch_tune(self.handle, int(reps),
                                          None if cache_path is None else os.fsencode(cache_path), byref(out),
                                          byref(ms), byref(hit)))
        return _schedule_dict(out), float(ms.value), bool(hit.value)

    def autotune(self, reps=2):
        choice = np.zeros(2, np.int32)
        ms = c_float()
        self._err(self.lib.mtp_batch_autotune(self.handle, int(reps), choice.ctypes.data_as(c_void_p), byref(ms)))
        return int(choice[0]), int(choice[1]), float(ms.value)


class mtp_completion(ctypes.Structure):
    _fields_ = [("ticket", c_uint64), ("robot", c_int32), ("status", c_int32), ("t_arrival_ns", c_uint64),
                ("t_admit_ns", c_uint64), ("t_done_ns", c_uint64), ("replan_idx", c_uint32), ("n", c_int32),
                ("u", c_float * 32)]


class mtp_server_stats(ctypes.Structure):
    _fields_ = [(name, c_uint64) for name in
                ("submitted", "admitted", "completed", "launches", "deferred_for_budget", "dropped", "pool_bytes",
                 "pool_in_use", "pool_peak", "resident_bytes")] + [("queued", c_int32), ("in_flight", c_int32),
                                                                   ("robots", c_int32), ("pad", c_int32)]


class Server:
    """Continuous-batching request loop over a fleet of robots (mtp_server).

    The server's device arena (launch tables and a pool of budget_bytes that
    holds the robots' resident buffers and the requests' transient slabs) is
    one torch allocation.  simulated=True drives the same scheduler with a
    host-only stand-in for the device (no GPU, zero actions, synthetic launch
    times).  Robots given as `robots` are added in order (ids 0, 1, ...)."""

    def __init__(self, budget_bytes, max_robots, iters_per_launch=1, max_inflight=2, device="cuda",
                 simulated=False, ns_per_sample_step=0.0, queue_items=0, robots=()):
        self.lib = load()
        self.cfgs = {}
        self._keep = {}
        h = c_void_p()
        self.workspace = None
        self.simulated = simulated
        if simulated:
            st = self.lib.mtp_server_create_simulated(int(budget_bytes), int(max_robots), int(queue_items),
                                                      int(iters_per_launch), int(max_inflight),
                                                      float(ns_per_sample_step), byref(h))
        else:
            torch = _torch()
            nbytes = int(self.lib.mtp_server_workspace_bytes(int(budget_bytes), int(max_robots), int(queue_items)))
            if nbytes == 0:
                raise MtpError(1, "server workspace size: invalid budget or robot count")
            self.device = torch.device(device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            st = self.lib.mtp_server_create(int(budget_bytes), int(max_robots), int(queue_items),
                                            int(iters_per_launch), int(max_inflight),
                                            c_void_p(self.workspace.data_ptr()), nbytes,
                                            c_void_p(self.stream.cuda_stream), byref(h))
        _check(self.lib, st)
        self.handle = h
        self._buf = (mtp_completion * 1024)()
        for c in robots:
            self.add_robot(c)

    def add_robot(self, cfg):
        c, keep = config_struct(cfg)
        rid = c_int32()
        self._err(self.lib.mtp_server_add_robot(self.handle, byref(c), byref(rid)))
        self.cfgs[int(rid.value)] = cfg
        return int(rid.value)

    def remove_robot(self, robot):
        self._err(self.lib.mtp_server_remove_robot(self.handle, int(robot)))
        self.cfgs.pop(int(robot), None)

    def robot_state(self, robot):
        """(mu, sigma) as (T, n) float32 device tensors and the next replan index."""
        torch = _torch()
        cfg = self.cfgs[int(robot)]
        mu = torch.empty((cfg.horizon, cfg.ctrl_dim), dtype=torch.float32, device=self.device)
        sg = torch.empty_like(mu)
        r = c_uint32()
        self._err(self.lib.mtp_server_get_robot_state(self.handle, int(robot), c_void_p(mu.data_ptr()),
                                                      c_void_p(sg.data_ptr()), byref(r)))
        return mu, sg, int(r.value)

    def _err(self, st):
        if st != 0:
            raise MtpError(st, self.lib.mtp_status_str(st).decode() + ": " +
                           self.lib.mtp_server_last_error(self.handle).decode())

    def now_ns(self):
        return int(self.lib.mtp_server_now_ns())

    def submit(self, robot, x0, shift=1, t_arrival_ns=None):
        x = np.ascontiguousarray(np.asarray(x0, np.float32))
        t = self.now_ns() if t_arrival_ns is None else int(t_arrival_ns)
        tk = c_uint64()
        self._err(self.lib.mtp_server_submit(self.handle, int(robot), x.ctypes.data_as(c_void_p), int(shift), t,
                                             byref(tk)))
        return int(tk.value)

    def pump(self, wait_us=0):
        n = c_int32()
        self._err(self.lib.mtp_server_pump(self.handle, int(wait_us), byref(n)))
        return int(n.value)

    def poll(self):
        out = []
        while True:
            n = c_int32()
            self._err(self.lib.mtp_server_poll(self.handle, self._buf, 1024, byref(n)))
            for i in range(n.value):
                c = self._buf[i]
                out.append(dict(ticket=int(c.ticket), robot=int(c.robot), status=int(c.status),
                                t_arrival_ns=int(c.t_arrival_ns), t_admit_ns=int(c.t_admit_ns),
                                t_done_ns=int(c.t_done_ns), replan_idx=int(c.replan_idx),
                                u=np.array(c.u[:c.n], np.float32)))
            if n.value < 1024:
                return out

    def stats(self):
        st = mtp_server_stats()
        self._err(self.lib.mtp_server_get_stats(self.handle, byref(st)))
        return {name: getattr(st, name) for name, _ in mtp_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mtp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
