"""MI355X-native two-belt pseudopotential lattice Boltzmann step (arXiv:1402.6019).

The compute path is the HIP library ``liblb355.so`` behind the C ABI of ``include/lb.h``;
``Sim`` is a thin wrapper that owns the device buffers as torch tensors (PyTorch is used for
device memory and streams only) and forwards every call to the library.
"""

import ctypes

import numpy as np

from . import _binding as B
from ._binding import LB_BF16DEV, LB_F32, LB_F64, LbError

STORAGE = {"f64": LB_F64, "f32": LB_F32, "bf16dev": LB_BF16DEV}

__all__ = ["Sim", "Batch", "LbError", "STORAGE", "default_weights", "fit_cooperative_length"]


def default_weights():
    """(w[5], p[5], t[2]) defaults of the library (isotropic sets, E2 = 1/3)."""
    c = B.default_couplings()
    return list(c.w), list(c.p), list(c.t)


def _pair(v):
    if np.isscalar(v):
        return (float(v), float(v))
    v = tuple(float(x) for x in v)
    return v if len(v) == 2 else (v[0], v[0])


def _couplings(g1=(0.0, 0.0), g2=(0.0, 0.0), gab=0.0, body=(0.0, 0.0), rho_wall=(0.0, 0.0), w=None, p=None, t=None,
               cross_psi=False, u_wall=(0.0, 0.0)):
    cpl = B.default_couplings()
    cpl.g1[:] = _pair(g1)
    cpl.g2[:] = _pair(g2)
    cpl.g_ab = float(gab)
    if w is not None:
        cpl.w[:] = [float(v) for v in w]
    if p is not None:
        cpl.p[:] = [float(v) for v in p]
    if t is not None:
        cpl.t[:] = [float(v) for v in t]
    cpl.body_force[:] = _pair(body) if len(body) == 2 else body
    cpl.rho_wall[:] = _pair(rho_wall)
    cpl.cross_uses_psi = 1 if cross_psi else 0
    cpl.wall_velocity[:] = tuple(float(v) for v in u_wall)
    return cpl


def _density(rho_init, ns, ly, lx):
    return np.ascontiguousarray(np.broadcast_to(rho_init, (ns, ly, lx)), dtype=np.float64)


def _psi_params(psi0, rho0, rho_ref, rho):
    if rho_ref is None:  # deviations from the mean initial density of each species
        rho_ref = tuple(float(r.mean()) for r in rho) + (0.0,) * (2 - rho.shape[0])
    return B.LbPsiParams(float(psi0), float(rho0), (ctypes.c_double * 2)(*_pair(rho_ref)))


class Sim:
    """One lattice on one GPU.

    Parameters follow the paper's statement of the problem: lattice (lx, ly, species,
    walls), couplings g1 = G_ss,1, g2 = G_ss,2, gab = G_AB, body force g, relaxation time
    tau, pseudopotential psi0 (1 - exp(-rho / rho0)); rho_init is the initial density
    [n_species, ly, lx] (host array), started from rest equilibrium.  rho_ref: reference
    density per species for the FP32/BF16 deviation storage (default: mean of rho_init).
    u_wall: x-velocities of the bottom and top walls (channel only; the planar Couette cell
    of the emulsion section moves them with -U_w and +U_w).
    """

    def __init__(self, lx, ly, rho_init, n_species=1, walls=False, storage="f64", g1=(0.0, 0.0),
                 g2=(0.0, 0.0), gab=0.0, body=(0.0, 0.0), rho_wall=(0.0, 0.0), tau=(1.0, 1.0), psi0=1.0,
                 rho0=1.0, rho_ref=None, w=None, p=None, t=None, cross_psi=False, device="cuda",
                 tile=None, u_wall=(0.0, 0.0)):
        import torch
        self._lib = B.load()
        self.torch = torch
        self.device = torch.device(device)
        self.lx, self.ly, self.ns = int(lx), int(ly), int(n_species)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.lat = B.LbLattice(self.lx, self.ly, self.ns, 1 if walls else 0, self.storage)
        cpl = _couplings(g1, g2, gab, body, rho_wall, w, p, t, cross_psi, u_wall)
        self.cpl = cpl
        self._ckw = dict(g1=g1, g2=g2, gab=gab, body=body, rho_wall=rho_wall, w=w, p=p, t=t, cross_psi=cross_psi,
                         u_wall=u_wall)
        self.tau = (ctypes.c_double * 2)(*_pair(tau))
        rho = _density(rho_init, self.ns, self.ly, self.lx)
        self.psi = _psi_params(psi0, rho0, rho_ref, rho)
        nbytes = B.pop_bytes(self.lat)
        if nbytes == 0:
            raise LbError(B.LB_EINVAL, "invalid lattice")
        self.pop_bytes = nbytes
        self.pop_a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.pop_b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self._lib.lb_init(ctypes.byref(h), ctypes.byref(self.lat), ctypes.byref(cpl), self.tau,
                               ctypes.byref(self.psi), rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.c_void_p(self.pop_a.data_ptr()), ctypes.c_void_p(self.pop_b.data_ptr()),
                               nbytes, ctypes.c_void_p(self.stream.cuda_stream))
        B.check(rc, None)
        self._h = h
        if tile is not None:
            self.set_tile(*tile)

    # -- lifetime -------------------------------------------------------------------------
    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lb_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        return B.check(rc, self._h)

    # -- C ABI ----------------------------------------------------------------------------
    @property
    def time(self):
        return self._lib.lb_time(self._h)

    def set_time(self, t):
        """Set the step count (resuming a checkpointed run in a new context)."""
        self._chk(self._lib.lb_set_time(self._h, int(t)))

    def set_two_step(self, enable=True, rows=0):
        """Advance plain steps two per launch (bitwise the same results): True, False or "auto"
        (the default: pairs for walled FP32 and periodic FP64 lattices beyond the Infinity
        Cache)."""
        mode = 2 if enable == "auto" else (1 if enable else 0)
        self._chk(self._lib.lb_set_two_step(self._h, mode, int(rows)))

    @property
    def two_step_active(self):
        """Whether step() currently advances plain steps two per launch."""
        return self._lib.lb_two_step_active(self._h) == 1

    def step(self, n=1):
        self._chk(self._lib.lb_step(self._h, int(n)))

    def set_reduce_every(self, k):
        self._chk(self._lib.lb_set_reduce_every(self._h, int(k)))

    def set_tile(self, tx, sy):
        self._chk(self._lib.lb_set_tile(self._h, int(tx), int(sy)))

    ROUNDINGS = {"nearest": 0, "stochastic": 1}

    def set_rounding(self, mode):
        """Rounding of the BF16 population stores: "nearest" (default) or "stochastic"
        (unbiased, reproducible; keeps increments far below one BF16 step on average)."""
        if mode not in self.ROUNDINGS:
            raise ValueError(f"mode must be one of {sorted(self.ROUNDINGS)}")
        self._chk(self._lib.lb_set_rounding(self._h, self.ROUNDINGS[mode]))

    STORE_POLICIES = {"auto": 0, "write_through": 1, "streaming": 2}

    def set_store_policy(self, policy):
        """Step-kernel variant for the population traffic: "auto" (by footprint),
        "write_through" or "streaming"; bitwise the same results, different speed."""
        if policy not in self.STORE_POLICIES:
            raise ValueError(f"policy must be one of {sorted(self.STORE_POLICIES)}")
        self._chk(self._lib.lb_set_store_policy(self._h, self.STORE_POLICIES[policy]))

    def get_tile(self):
        tx, sy = ctypes.c_int32(), ctypes.c_int32()
        self._chk(self._lib.lb_get_tile(self._h, ctypes.byref(tx), ctypes.byref(sy)))
        return tx.value, sy.value

    def set_couplings(self, **kw):
        """Replace couplings (any of g1, g2, gab, body, rho_wall, w, p, t, cross_psi, u_wall);
        the others keep their current values."""
        self._ckw.update(kw)
        cpl = _couplings(**self._ckw)
        self._chk(self._lib.lb_set_couplings(self._h, ctypes.byref(cpl)))
        self.cpl = cpl

    def adjoint(self, T, loss_weights=(1.0, 0.0), every=0, fp64_reverse=False):
        """Loss L = lw0 <(W_bot + W_top)/2> + lw1 <Q> over the next T steps and its gradient
        dL/d(G_AA,1, G_BB,1, G_AA,2, G_BB,2, G_AB, g_x, g_y) by the hand-written adjoint with
        checkpoints every `every` steps (0: sqrt(T); 1: no checkpoints, the forward pass keeps
        what the reverse step reads of every state, about T x 64 B per site with an FP64
        reverse sweep, and nothing is recomputed); fp64_reverse runs the reverse sweep in FP64
        for FP32 / BF16 storage.  Advances the state by T steps."""
        torch = self.torch
        flags = B.LB_ADJ_FP64 if fp64_reverse else 0
        nbytes = self._lib.lb_adjoint_workspace_bytes(self._h, int(T), int(every), flags)
        if nbytes == 0:
            raise LbError(B.LB_EINVAL, "invalid adjoint request")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        lw = (ctypes.c_double * 2)(*[float(v) for v in loss_weights])
        loss = ctypes.c_double()
        grad = (ctypes.c_double * 7)()
        self._chk(self._lib.lb_adjoint(self._h, int(T), int(every), flags, lw, ctypes.byref(loss), grad,
                                       ctypes.c_void_p(ws.data_ptr()), nbytes))
        del ws
        return loss.value, np.array(grad[:])

    def set_graph(self, steps):
        """Replay plain steps in captured HIP graphs of `steps` launches (0: off)."""
        self._chk(self._lib.lb_set_graph(self._h, int(steps)))

    def autotune(self, trial_steps=20):
        """Pick the fastest launch shape by timing; returns ((tx, sy), ms per step)."""
        tx, sy, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._chk(self._lib.lb_autotune(self._h, int(trial_steps), ctypes.byref(tx), ctypes.byref(sy), ctypes.byref(ms)))
        return (tx.value, sy.value), ms.value

    def moments(self, dtype=None):
        """(rho [ns, ly, lx], u [2, ly, lx]) device tensors of the current state."""
        torch = self.torch
        dtype = dtype or torch.float64
        rho = torch.empty((self.ns, self.ly, self.lx), dtype=dtype, device=self.device)
        u = torch.empty((2, self.ly, self.lx), dtype=dtype, device=self.device)
        code = B.LB_OUT_F32 if dtype == torch.float32 else B.LB_OUT_F64
        self._chk(self._lib.lb_moments(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()), code))
        return rho, u

    def totals(self):
        """(mass[2], momentum[2], flow) of the current state (FP64; synchronises)."""
        m = (ctypes.c_double * 2)()
        p = (ctypes.c_double * 2)()
        q = ctypes.c_double()
        self._chk(self._lib.lb_totals(self._h, m, p, ctypes.byref(q)))
        return (m[0], m[1]), (p[0], p[1]), q.value

    def wall_stress(self, reset=False):
        out = (ctypes.c_double * 2)()
        self._chk(self._lib.lb_wall_stress(self._h, out, 1 if reset else 0))
        return out[0], out[1]

    def stress_field(self, dtype=None):
        """Site pressure tensor of the current state (Appendix A): device tensor [3, ly, lx]
        with the xx, xy and yy components."""
        torch = self.torch
        dtype = dtype or torch.float64
        out = torch.empty((3, self.ly, self.lx), dtype=dtype, device=self.device)
        code = B.LB_OUT_F32 if dtype == torch.float32 else B.LB_OUT_F64
        self._chk(self._lib.lb_stress_field(self._h, ctypes.c_void_p(out.data_ptr()), code))
        return out

    def profile(self, out=None):
        """Stream-wise averaged profiles of the current state (device FP64 tensor of 4 ly + 1):
        [0:ly] the x-averaged velocity ubar(y), [ly:2ly+1] the shear stress sigma(k) through
        the lines k = 0..ly between rows k-1 and k (sigma(0) = W_bot, sigma(ly) = -W_top on a
        channel), [2ly+1:3ly+1] and [3ly+1:] the x-averaged densities of species A and B."""
        torch = self.torch
        if out is None:
            out = torch.empty(4 * self.ly + 1, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != 4 * self.ly + 1:
            raise ValueError("out must be a contiguous float64 tensor of 4 ly + 1 elements")
        self._chk(self._lib.lb_profile(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def sample_profiles(self, n, every):
        """n profiles, one after every `every` steps (advances n * every steps): [n, 4 ly + 1]."""
        torch = self.torch
        out = torch.empty((int(n), 4 * self.ly + 1), dtype=torch.float64, device=self.device)
        for i in range(int(n)):
            self.step(every)
            self.profile(out[i])
        return out

    def profile_stats(self, samples, k0=None):
        """Time statistics of profile samples [n, 4 ly + 1]: dict of <ubar> [ly], <sigma> [ly+1],
        the time-averaged local fluidity <f> [ly+1], the stress correlator C_sigma(k, k0)
        [ly+1] (k0 default: the centre line) and the species densities <rho_A>, <rho_B> [ly]."""
        torch = self.torch
        ly = self.ly
        samples = samples.to(dtype=torch.float64, device=self.device).contiguous()
        if samples.dim() != 2 or samples.shape[1] != 4 * ly + 1:
            raise ValueError("samples must have shape (n, 4 ly + 1)")
        k0 = ly // 2 if k0 is None else int(k0)
        out = torch.empty(6 * ly + 3, dtype=torch.float64, device=self.device)
        self._chk(self._lib.lb_profile_stats(self._h, ctypes.c_void_p(samples.data_ptr()), samples.shape[0], k0,
                                             ctypes.c_void_p(out.data_ptr())))
        return dict(u=out[:ly], sigma=out[ly:2 * ly + 1], fluidity=out[2 * ly + 1:3 * ly + 2],
                    corr=out[3 * ly + 2:4 * ly + 3], rho_a=out[4 * ly + 3:5 * ly + 3], rho_b=out[5 * ly + 3:])

    def checkpoint(self):
        """Canonical FP64 pre-collision populations f[ns, 9, ly, lx] (device tensor)."""
        f = self.torch.empty((self.ns, 9, self.ly, self.lx), dtype=self.torch.float64, device=self.device)
        self._chk(self._lib.lb_checkpoint(self._h, ctypes.c_void_p(f.data_ptr())))
        return f

    def restore(self, f):
        f = self.torch.as_tensor(f, dtype=self.torch.float64, device=self.device).contiguous()
        if tuple(f.shape) != (self.ns, 9, self.ly, self.lx):
            raise ValueError("populations must have shape (n_species, 9, ly, lx)")
        self._keep = f  # keep alive until the asynchronous restore kernel has read it
        self._chk(self._lib.lb_restore(self._h, ctypes.c_void_p(f.data_ptr())))


def fit_cooperative_length(z, f, H, zeta_range=None):
    """Least-squares fit of eq. (predict) to a fluidity profile f(z), 0 <= z <= H:
    f = f_b + (f_w - f_b) cosh((z - H/2)/zeta) / cosh(H/(2 zeta)).  Returns
    dict(zeta, f_b, f_w, rms).  zeta_range: search interval (default (H/1000, 100 H))."""
    lib = B.load()
    z = np.ascontiguousarray(z, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    if z.shape != f.shape or z.ndim != 1:
        raise ValueError("z and f must be 1-D arrays of the same length")
    lo, hi = zeta_range if zeta_range is not None else (H / 1000.0, 100.0 * H)
    out = (ctypes.c_double * 4)()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.lb_fit_cooperative_length(z.ctypes.data_as(dp), f.ctypes.data_as(dp), len(z), float(H), float(lo),
                                       float(hi), out)
    if rc != B.LB_OK:
        raise LbError(rc, "invalid fit input")
    return dict(zeta=out[0], f_b=out[1], f_w=out[2], rms=out[3])


class Batch:
    """Many independent lattices stepped together by one persistent launch per time step.

    instances: list of dicts with the keyword arguments of Sim (lx, ly, rho_init, and any of
    g1, g2, gab, body, rho_wall, tau, psi0, rho0, rho_ref, w, p, t, cross_psi, u_wall); storage,
    n_species and walls are common to all instances.
    """

    def __init__(self, instances, n_species=2, walls=True, storage="f32", device="cuda"):
        import torch
        self._lib = B.load()
        self.torch = torch
        self.device = torch.device(device)
        self.n = len(instances)
        self.ns = int(n_species)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        n = self.n
        self.lats = (B.LbLattice * n)()
        self.cpls = (B.LbCouplings * n)()
        self.psis = (B.LbPsiParams * n)()
        self.taus = (ctypes.c_double * (2 * n))()
        self._rho = []
        self.shapes = []
        for i, inst in enumerate(instances):
            lx, ly = int(inst["lx"]), int(inst["ly"])
            self.shapes.append((lx, ly))
            self.lats[i] = B.LbLattice(lx, ly, self.ns, 1 if walls else 0, self.storage)
            self.cpls[i] = _couplings(inst.get("g1", (0.0, 0.0)), inst.get("g2", (0.0, 0.0)), inst.get("gab", 0.0),
                                      inst.get("body", (0.0, 0.0)), inst.get("rho_wall", (0.0, 0.0)), inst.get("w"),
                                      inst.get("p"), inst.get("t"), inst.get("cross_psi", False),
                                      inst.get("u_wall", (0.0, 0.0)))
            tau = _pair(inst.get("tau", (1.0, 1.0)))
            self.taus[2 * i], self.taus[2 * i + 1] = tau
            rho = _density(inst["rho_init"], self.ns, ly, lx)
            self._rho.append(rho)
            self.psis[i] = _psi_params(inst.get("psi0", 1.0), inst.get("rho0", 1.0), inst.get("rho_ref"), rho)
        nbytes = self._lib.lb_batch_pop_bytes(n, self.lats)
        if nbytes == 0:
            raise LbError(B.LB_EINVAL, "invalid lattice in batch")
        self.pop_bytes = nbytes
        self.pop_a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.pop_b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ptrs = (ctypes.POINTER(ctypes.c_double) * n)(*[r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                                        for r in self._rho])
        h = ctypes.c_void_p()
        rc = self._lib.lb_batch_init(ctypes.byref(h), n, self.lats, self.cpls, self.taus, self.psis, ptrs,
                                     ctypes.c_void_p(self.pop_a.data_ptr()), ctypes.c_void_p(self.pop_b.data_ptr()),
                                     nbytes, ctypes.c_void_p(self.stream.cuda_stream))
        B.check_batch(rc, None)
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lb_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        return B.check_batch(rc, self._h)

    @property
    def time(self):
        return self._lib.lb_batch_time(self._h)

    def set_time(self, t):
        """Set the common step count (resuming checkpointed instances in a new batch)."""
        self._chk(self._lib.lb_batch_set_time(self._h, int(t)))

    def step(self, n=1):
        self._chk(self._lib.lb_batch_step(self._h, int(n)))

    def set_reduce_every(self, k):
        self._chk(self._lib.lb_batch_set_reduce_every(self._h, int(k)))

    def set_graph(self, steps):
        self._chk(self._lib.lb_batch_set_graph(self._h, int(steps)))

    def set_rounding(self, mode):
        """Rounding of every instance's BF16 population stores: "nearest" or "stochastic"."""
        if mode not in Sim.ROUNDINGS:
            raise ValueError(f"mode must be one of {sorted(Sim.ROUNDINGS)}")
        self._chk(self._lib.lb_batch_set_rounding(self._h, Sim.ROUNDINGS[mode]))

    def set_tile(self, tx, sy, grid=0):
        self._chk(self._lib.lb_batch_set_tile(self._h, int(tx), int(sy), int(grid)))

    def get_tile(self):
        tx, sy, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._chk(self._lib.lb_batch_get_tile(self._h, ctypes.byref(tx), ctypes.byref(sy), ctypes.byref(g)))
        return tx.value, sy.value, g.value

    def autotune(self, trial_steps=10):
        out = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double()
        self._chk(self._lib.lb_batch_autotune(self._h, int(trial_steps), out, ctypes.byref(ms)))
        return tuple(out), ms.value

    def moments(self, i, dtype=None):
        torch = self.torch
        dtype = dtype or torch.float64
        lx, ly = self.shapes[i]
        rho = torch.empty((self.ns, ly, lx), dtype=dtype, device=self.device)
        u = torch.empty((2, ly, lx), dtype=dtype, device=self.device)
        code = B.LB_OUT_F32 if dtype == torch.float32 else B.LB_OUT_F64
        self._chk(self._lib.lb_batch_moments(self._h, int(i), ctypes.c_void_p(rho.data_ptr()),
                                             ctypes.c_void_p(u.data_ptr()), code))
        return rho, u

    def profile(self, i):
        """Profiles of instance i (device FP64 [4 ly_i + 1]), as Sim.profile."""
        torch = self.torch
        lx, ly = self.shapes[i]
        out = torch.empty(4 * ly + 1, dtype=torch.float64, device=self.device)
        self._chk(self._lib.lb_batch_profile(self._h, int(i), ctypes.c_void_p(out.data_ptr())))
        return out

    def stress_field(self, i, dtype=None):
        """Site pressure tensor of instance i (device [3, ly_i, lx_i]), as Sim.stress_field."""
        torch = self.torch
        dtype = dtype or torch.float64
        lx, ly = self.shapes[i]
        out = torch.empty((3, ly, lx), dtype=dtype, device=self.device)
        code = B.LB_OUT_F32 if dtype == torch.float32 else B.LB_OUT_F64
        self._chk(self._lib.lb_batch_stress_field(self._h, int(i), ctypes.c_void_p(out.data_ptr()), code))
        return out

    def totals(self):
        """[n, 5] FP64: mass A, mass B, momentum x, momentum y, flow rate."""
        out = np.zeros((self.n, 5))
        self._chk(self._lib.lb_batch_totals(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def wall_stress(self, reset=False):
        out = np.zeros((self.n, 2))
        self._chk(self._lib.lb_batch_wall_stress(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 1 if reset else 0))
        return out

    def checkpoint(self, i):
        lx, ly = self.shapes[i]
        f = self.torch.empty((self.ns, 9, ly, lx), dtype=self.torch.float64, device=self.device)
        self._chk(self._lib.lb_batch_checkpoint(self._h, int(i), ctypes.c_void_p(f.data_ptr())))
        return f

    def restore(self, i, f):
        lx, ly = self.shapes[i]
        f = self.torch.as_tensor(f, dtype=self.torch.float64, device=self.device).contiguous()
        if tuple(f.shape) != (self.ns, 9, ly, lx):
            raise ValueError("populations must have shape (n_species, 9, ly, lx)")
        self._keep = f
        self._chk(self._lib.lb_batch_restore(self._h, int(i), ctypes.c_void_p(f.data_ptr())))


class Sim3:
    """One 3-D lattice (D3Q19, include/lb3.h) on one GPU: the two-belt force over the 5x5x5
    cube, one or two species, periodic or bounded in y by bounce-back walls.  rho_init:
    [n_species, lz, ly, lx] host array; the state starts at rest.  Storage "f64" or "f32"."""

    def __init__(self, lx, ly, lz, rho_init, n_species=1, walls=False, storage="f64", g1=(0.0, 0.0),
                 g2=(0.0, 0.0), gab=0.0, body=(0.0, 0.0, 0.0), rho_wall=(0.0, 0.0), tau=(1.0, 1.0), psi0=1.0,
                 rho0=1.0, rho_ref=None, w=None, p=None, t=None, cross_psi=False, device="cuda", tile=None):
        import torch
        self._lib = B.load()
        self.torch = torch
        self.device = torch.device(device)
        self.lx, self.ly, self.lz, self.ns = int(lx), int(ly), int(lz), int(n_species)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.lat = B.Lb3Lattice(self.lx, self.ly, self.lz, self.ns, 1 if walls else 0, self.storage)
        c = B.Lb3Couplings()
        B.check3(self._lib.lb3_default_couplings(ctypes.byref(c)))
        g1, g2, rw = _pair(g1), _pair(g2), _pair(rho_wall)
        for k in range(2):
            c.g1[k], c.g2[k], c.rho_wall[k] = g1[k], g2[k], rw[k]
        c.g_ab = float(gab)
        for k in range(3):
            c.body_force[k] = float(body[k])
        if w is not None:
            for q in range(7):
                c.w[q] = float(w[q])
        if p is not None:
            for q in range(7):
                c.p[q] = float(p[q])
        if t is not None:
            c.t[0], c.t[1] = float(t[0]), float(t[1])
        c.cross_uses_psi = 1 if cross_psi else 0
        self.cpl = c
        self.tau = (ctypes.c_double * 2)(*_pair(tau))
        rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho_init, dtype=np.float64),
                                                   (self.ns, self.lz, self.ly, self.lx)))
        ref = rho_ref if rho_ref is not None else tuple(float(rho[s].mean()) for s in range(self.ns))
        self.psi = B.LbPsiParams(float(psi0), float(rho0), (ctypes.c_double * 2)(*_pair(ref)))
        nbytes = self._lib.lb3_pop_bytes(ctypes.byref(self.lat))
        if nbytes == 0:
            raise LbError(B.LB_EINVAL, "invalid 3-D lattice")
        self.pop_bytes = nbytes
        self.pop_a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.pop_b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self._lib.lb3_init(ctypes.byref(h), ctypes.byref(self.lat), ctypes.byref(c), self.tau,
                                ctypes.byref(self.psi), rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.c_void_p(self.pop_a.data_ptr()), ctypes.c_void_p(self.pop_b.data_ptr()),
                                nbytes, ctypes.c_void_p(self.stream.cuda_stream))
        B.check3(rc, None)
        self._h = h
        if tile is not None:
            self.set_tile(*tile)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lb3_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        return B.check3(rc, self._h)

    @property
    def time(self):
        return self._lib.lb3_time(self._h)

    def step(self, n=1):
        self._chk(self._lib.lb3_step(self._h, int(n)))

    def set_tile(self, ty, sz):
        self._chk(self._lib.lb3_set_tile(self._h, int(ty), int(sz)))

    def get_tile(self):
        ty, sz = ctypes.c_int32(), ctypes.c_int32()
        self._chk(self._lib.lb3_get_tile(self._h, ctypes.byref(ty), ctypes.byref(sz)))
        return ty.value, sz.value

    def moments(self, dtype=None):
        """(rho [ns, lz, ly, lx], u [3, lz, ly, lx]) device tensors of the current state."""
        torch = self.torch
        dtype = dtype or torch.float64
        rho = torch.empty((self.ns, self.lz, self.ly, self.lx), dtype=dtype, device=self.device)
        u = torch.empty((3, self.lz, self.ly, self.lx), dtype=dtype, device=self.device)
        code = B.LB_OUT_F32 if dtype == torch.float32 else B.LB_OUT_F64
        self._chk(self._lib.lb3_moments(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()), code))
        return rho, u

    def totals(self):
        """(mass[2], momentum[3], flow) of the current state (FP64; synchronises)."""
        m, p, q = (ctypes.c_double * 2)(), (ctypes.c_double * 3)(), ctypes.c_double()
        self._chk(self._lib.lb3_totals(self._h, m, p, ctypes.byref(q)))
        return list(m), list(p), q.value

    def checkpoint(self):
        """Canonical FP64 pre-collision populations f[ns, 19, lz, ly, lx] (device tensor)."""
        f = self.torch.empty((self.ns, 19, self.lz, self.ly, self.lx), dtype=self.torch.float64, device=self.device)
        self._chk(self._lib.lb3_checkpoint(self._h, ctypes.c_void_p(f.data_ptr())))
        return f

    def restore(self, f):
        f = self.torch.as_tensor(f, dtype=self.torch.float64, device=self.device).contiguous()
        if tuple(f.shape) != (self.ns, 19, self.lz, self.ly, self.lx):
            raise ValueError("populations must have shape (n_species, 19, lz, ly, lx)")
        self._keep = f
        self._chk(self._lib.lb3_restore(self._h, ctypes.c_void_p(f.data_ptr())))
