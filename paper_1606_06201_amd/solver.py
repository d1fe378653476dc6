"""Python front end of libipmg: one Solver per grid, torch tensors for device
memory and the current HIP stream.  Every numerical step runs in the library's
kernels; this module only checks arguments and passes pointers."""
import ctypes as C

import numpy as np
import torch

from . import _lib as L

OP_K, OP_Z = L.OP_K, L.OP_Z


class IPMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ipmg error {code}: {msg}")
        self.code = code


class Solver:
    """Multigrid-preconditioned CG on K(x) (and the interior-point augmented
    system Z) for a structured Q1 grid of nel = (nx, ny[, nz]) unit elements."""

    def __init__(self, nel, levels, fp32=True, E=1.0, nu=0.3, nu_pre=2, nu_post=2, omega=0.6,
                 flexible=False, device="cuda:0"):
        self.lib = L.load()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the ipmg library runs on a GPU device")
        nel = tuple(int(v) for v in nel)
        d = L.Desc()
        d.dim = len(nel)
        for a in range(3):
            d.nel[a] = nel[a] if a < len(nel) else 1
        d.levels, d.E, d.nu = int(levels), float(E), float(nu)
        d.vcycle_fp32, d.nu_pre, d.nu_post, d.omega = int(bool(fp32)), int(nu_pre), int(nu_post), float(omega)
        d.pcg_flexible = int(bool(flexible))
        self.nel, self.dim, self.levels, self.fp32 = nel, len(nel), int(levels), bool(fp32)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            rc = self.lib.ipmg_create(C.byref(d), C.c_void_p(stream), C.byref(h))
        if rc != L.OK:
            raise IPMGError(rc, self.lib.ipmg_status_string(rc).decode())
        self.h = h
        self.n_slots, self.n_free, self.m = self.sizes(levels - 1)

    # -------------------------------------------------------------- plumbing --
    def close(self):
        if getattr(self, "h", None):
            self.lib.ipmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != L.OK and rc not in allow:
            msg = self.lib.ipmg_last_error(self.h).decode()
            raise IPMGError(rc, msg or self.lib.ipmg_status_string(rc).decode())
        return rc

    def _ptr(self, t, n, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != n:
            raise ValueError(f"{name} must have {n} entries, got {t.numel()}")
        return C.c_void_p(t.data_ptr())

    def _empty(self, n):
        return torch.empty(n, dtype=torch.float64, device=self.device)

    def _zeros(self, n):
        return torch.zeros(n, dtype=torch.float64, device=self.device)

    def _call(self, fn, *args, allow=()):
        with torch.cuda.device(self.device):
            return self._check(fn(self.h, *args), allow)

    def _n(self, op):
        return self.n_slots + (1 if op == OP_Z else 0)

    # ------------------------------------------------------------- integer maps --
    def sizes(self, level):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.ipmg_sizes(self.h, int(level), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def dof_map(self, level):
        n_free = self.sizes(level)[1]
        out = np.empty(n_free, dtype=np.int64)
        self._check(self.lib.ipmg_dof_map(self.h, int(level), out.ctypes.data_as(C.c_void_p)))
        return out

    def slot_of(self, level, i, j, k=0, c=0):
        return int(self.lib.ipmg_slot_of(self.h, int(level), int(i), int(j), int(k), int(c)))

    def load_vector(self, loads):
        """Slot vector from [(node coords, component, value)] point loads."""
        f = np.zeros(self.n_slots)
        for coords, comp, val in loads:
            coords = tuple(coords) + (0,) * (3 - len(coords))
            s = self.slot_of(self.levels - 1, coords[0], coords[1], coords[2], comp)
            if s < 0:
                raise ValueError(f"load outside the grid: {coords}")
            f[s] += val
        return torch.from_numpy(f).to(self.device)

    def element_matrix(self):
        nd = self.dim * 2 ** self.dim
        out = np.empty((nd, nd))
        self._check(self.lib.ipmg_element_matrix(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    # ---------------------------------------------------------------- operators --
    def set_density(self, x):
        self._call(self.lib.ipmg_set_density, self._ptr(x, self.m, "x"))

    def apply_K(self, v, out=None):
        out = self._empty(self.n_slots) if out is None else out
        self._call(self.lib.ipmg_apply_K, self._ptr(v, self.n_slots, "v"), self._ptr(out, self.n_slots, "y"))
        return out

    def apply_Z(self, v, out=None):
        n = self.n_slots + 1
        out = self._empty(n) if out is None else out
        self._call(self.lib.ipmg_apply_Z, self._ptr(v, n, "v"), self._ptr(out, n, "y"))
        return out

    def mg_setup(self, op=OP_K):
        self._call(self.lib.ipmg_mg_setup, int(op))

    def level_damping(self, level):
        """(omega_k, rho_k) of the Jacobi smoother on a level after mg_setup."""
        w, r = C.c_double(), C.c_double()
        self._call(self.lib.ipmg_level_damping, int(level), C.byref(w), C.byref(r))
        return w.value, r.value

    def vcycle(self, r, op=OP_K, out=None):
        n = self._n(op)
        out = self._empty(n) if out is None else out
        self._call(self.lib.ipmg_vcycle, int(op), self._ptr(r, n, "r"), self._ptr(out, n, "z"))
        return out

    def pcg(self, b, op=OP_K, u0=None, rtol=1e-8, maxit=1000, check=True):
        """Solve A u = b by MG-PCG; returns (u, info dict)."""
        n = self._n(op)
        u = self._zeros(n) if u0 is None else u0.clone()
        info = L.PCGInfo()
        allow = () if check else (L.E_NOT_CONVERGED, L.E_BREAKDOWN)
        rc = self._call(self.lib.ipmg_pcg, int(op), self._ptr(b, n, "b"), self._ptr(u, n, "u"),
                        float(rtol), int(maxit), C.byref(info), allow=allow)
        return u, dict(iters=info.iters, restarts=info.restarts, status=info.status, relres=info.relres,
                       true_relres=info.true_relres, setup_ms=info.setup_ms, solve_ms=info.solve_ms, bu=info.bu,
                       rc=rc)

    def pcg_noalloc(self, b, op=OP_K, u0=None, rtol=1e-8, maxit=1000, check=True):
        """pcg through ipmg_pcg_noalloc: the library's static scratch array instead of
        the context's work vectors (the hierarchy of op must be set up already)."""
        n = self._n(op)
        u = self._zeros(n) if u0 is None else u0.clone()
        info = L.PCGInfo()
        allow = () if check else (L.E_NOT_CONVERGED, L.E_BREAKDOWN)
        rc = self._call(self.lib.ipmg_pcg_noalloc, int(op), self._ptr(b, n, "b"), self._ptr(u, n, "u"),
                        float(rtol), int(maxit), C.byref(info), allow=allow)
        return u, dict(iters=info.iters, restarts=info.restarts, status=info.status, relres=info.relres,
                       true_relres=info.true_relres, setup_ms=info.setup_ms, solve_ms=info.solve_ms, bu=info.bu,
                       rc=rc)

    def pcg_noalloc_bytes(self):
        return int(self.lib.ipmg_pcg_noalloc_bytes(self.h))

    def element_sens(self, w, u, scale=1.0, out=None):
        out = self._empty(self.m) if out is None else out
        self._call(self.lib.ipmg_element_sens, self._ptr(w, self.n_slots, "w"), self._ptr(u, self.n_slots, "u"),
                   float(scale), self._ptr(out, self.m, "g"))
        return out

    # ------------------------------------------------------------------ SIMP --
    def filter(self, v, rmin=2.0, transpose=False, out=None):
        """Density filter of the SIMP model (Sec. 9): W v, or W' v."""
        out = self._empty(self.m) if out is None else out
        self._call(self.lib.ipmg_filter, float(rmin), self._ptr(v, self.m, "in"), self._ptr(out, self.m, "out"),
                   int(bool(transpose)))
        return out

    def simp_compliance(self, x, f, rmin=2.0, p=3.0, rtol=1e-8, maxit=1000):
        """(u, gradient, info) of the SIMP compliance at x (Sec. 9); info["bu"] = f'u."""
        u, grad = self._empty(self.n_slots), self._empty(self.m)
        info = L.PCGInfo()
        rc = self._call(self.lib.ipmg_simp_compliance, self._ptr(x, self.m, "x"), self._ptr(f, self.n_slots, "f"),
                        float(rmin), float(p), float(rtol), int(maxit), self._ptr(u, self.n_slots, "u"),
                        self._ptr(grad, self.m, "grad"), C.byref(info))
        return u, grad, dict(iters=info.iters, status=info.status, true_relres=info.true_relres, bu=info.bu, rc=rc)

    # ------------------------------------------------------------------- OC --
    def oc_update(self, u, x, V, xbar, q=1.0, lam_hi=1e4, tau=1e-11, blend=None, out=None):
        """One density update of Algorithm OC (q = 1) / DOC (q < 1), Sec. 4, with the
        device bisection for lambda; blend: AOC mean (blend + update) / 2.
        Returns (x_new, info dict)."""
        out = self._empty(self.m) if out is None else out
        info = L.OCInfo()
        bl = None if blend is None else self._ptr(blend, self.m, "blend")
        self._call(self.lib.ipmg_oc_update, self._ptr(u, self.n_slots, "u"), self._ptr(x, self.m, "x"),
                   float(V), float(xbar), float(q), float(lam_hi), float(tau), bl, self._ptr(out, self.m, "x_new"),
                   C.byref(info))
        return out, dict(lam=info.lam, volume=info.volume, trials=info.trials)

    def oc_run(self, f, x0, V, xbar, variant="oc", q=0.5, tau_oc=1e-5, cg_tol=1e-4, max_outer=10000,
               lam_hi=1e4, tau_lam=1e-11, maxit=1000):
        """Algorithm OC / DOC / AOC (Sec. 4) with the multigrid CG of Sec. 6.2: stop when
        |f'u_k - f'u_{k-1}| <= tau_oc (eq. (OCstop)); the relative tolerance of the
        solves starts at cg_tol and is multiplied by 0.1 whenever the compliance
        increases.  AOC: x1 = OC(x), x2 = OC(x1), x = (x1 + x2)/2.  Returns (x, u, log);
        log["feval"] counts the linear systems solved."""
        qq = q if variant == "doc" else 1.0
        x = x0.clone()
        log = dict(outer=0, feval=0, pcg_iters=[], compliance=[], cg_tol=[], lam=[], status="max_outer")
        tol = [float(cg_tol)]

        def solve_at(y):
            self.set_density(y)
            u, inf = self.pcg(f, rtol=tol[0], maxit=maxit)
            log["feval"] += 1
            log["pcg_iters"].append(inf["iters"])
            return u, inf["bu"]

        u, c_prev = solve_at(x)
        log["compliance"].append(c_prev)
        while log["outer"] < max_outer:
            if variant == "aoc":
                x1, _ = self.oc_update(u, x, V, xbar, 1.0, lam_hi, tau_lam)
                u1, _ = solve_at(x1)
                x, oi = self.oc_update(u1, x1, V, xbar, 1.0, lam_hi, tau_lam, blend=x1, out=x)
            else:
                x, oi = self.oc_update(u, x, V, xbar, qq, lam_hi, tau_lam, out=torch.empty_like(x))
            u, c = solve_at(x)
            log["outer"] += 1
            log["compliance"].append(c)
            log["lam"].append(oi["lam"])
            log["cg_tol"].append(tol[0])
            if c > c_prev:
                tol[0] *= 0.1
            if abs(c - c_prev) <= tau_oc:
                log["status"] = "converged"
                break
            c_prev = c
        return x, u, log

    # ------------------------------------------------------------------ timing --
    KERNEL_CLASSES = {"fine_jacobi": 0, "dir_apply": 1, "fine_resid": 2, "pcg_update": 3, "sub_jacobi": 4,
                      "fine_jacobi0": 5, "fine_jacobi_beta": 6, "sub_down": 7, "sub_up": 8,
                      "fine_pjacobi": 11, "fine_jacobi2": 12, "elem3": 13,
                      "elem3_dir": 14}

    def profile_begin(self, kernels, max_launches=4096):
        """Time every launch of the named kernel classes (a name or a list)."""
        names = [kernels] if isinstance(kernels, str) else list(kernels)
        mask = 0
        for k in names:
            mask |= 1 << self.KERNEL_CLASSES[k]
        self._call(self.lib.ipmg_profile_begin, mask, int(max_launches))
        self._prof_cap = int(max_launches)

    def profile_end(self):
        """Per-launch durations (ms) recorded since profile_begin, grouped by class
        name: {name: array of durations in launch order}."""
        out = np.zeros(self._prof_cap)
        cls = np.full(self._prof_cap, -1, dtype=np.int32)
        n = C.c_int()
        self._call(self.lib.ipmg_profile_end, out.ctypes.data_as(C.c_void_p), cls.ctypes.data_as(C.c_void_p),
                   self._prof_cap, C.byref(n))
        inv = {v: k for k, v in self.KERNEL_CLASSES.items()}
        res = {}
        for k in np.unique(cls[: n.value]):
            res[inv[int(k)]] = out[: n.value][cls[: n.value] == k].copy()
        return res

    # ------------------------------------------------------------ interior point --
    @staticmethod
    def ip_params(V, xbar=1.0, sigma=0.2, tau_nwt=0.1, pcg_rtol=1e-8, pcg_maxit=1000, frac=0.9,
                  step_all_blocks=True, stop="kkt", kkt_tol=1e-6, tau_ip=1e-8, max_newton=300,
                  accept_rtol=1e-2):
        p = L.IPParams()
        p.V, p.xbar, p.sigma, p.tau_nwt = float(V), float(xbar), float(sigma), float(tau_nwt)
        p.pcg_rtol, p.pcg_maxit, p.frac = float(pcg_rtol), int(pcg_maxit), float(frac)
        p.step_all_blocks = int(bool(step_all_blocks))
        p.stop_rule = {"kkt": 0, "barrier": 1}[stop]
        p.kkt_tol, p.tau_ip, p.max_newton = float(kkt_tol), float(tau_ip), int(max_newton)
        p.accept_rtol = float(accept_rtol)
        return p

    @classmethod
    def ip_params_paper(cls, V, xbar=2.0, cg_tol=1e-2, tau_ip=1e-8):
        """The paper's own inexact settings (Sec. 3, Sec. 6.1, Sec. 7): every Newton
        system solved to the relative residual 1e-2 (eq. (cgstop)), tau_NWT = 0.1,
        sigma = 0.2, stop at max(s, r) <= tau_IP = 1e-8 (eq. (crit:ip)), xbar = 2."""
        return cls.ip_params(V, xbar, pcg_rtol=cg_tol, stop="barrier", tau_ip=tau_ip, accept_rtol=cg_tol)

    def new_ip_state(self):
        return dict(u=self._zeros(self.n_slots), x=self._zeros(self.m), phi=self._zeros(self.m),
                    psi=self._zeros(self.m), lam=0.0, s=0.0, r=0.0)

    def _state_struct(self, st):
        s = L.IPState()
        s.u = self._ptr(st["u"], self.n_slots, "u").value
        s.x = self._ptr(st["x"], self.m, "x").value
        s.phi = self._ptr(st["phi"], self.m, "phi").value
        s.psi = self._ptr(st["psi"], self.m, "psi").value
        s.lam, s.s, s.r = float(st["lam"]), float(st["s"]), float(st["r"])
        return s

    @staticmethod
    def _state_back(s, st):
        st["lam"], st["s"], st["r"] = s.lam, s.s, s.r

    def ip_init(self, f, params, state=None, simp=None):
        """Starting point of the interior-point method; simp=(rmin, p): the SIMP model
        with the density filter (Sec. 9)."""
        st = self.new_ip_state() if state is None else state
        s = self._state_struct(st)
        info = L.PCGInfo()
        if simp is None:
            self._call(self.lib.ipmg_ip_init, self._ptr(f, self.n_slots, "f"), C.byref(params), C.byref(s),
                       C.byref(info))
        else:
            self._call(self.lib.ipmg_simp_ip_init, self._ptr(f, self.n_slots, "f"), C.byref(params),
                       float(simp[0]), float(simp[1]), C.byref(s), C.byref(info))
        self._state_back(s, st)
        return st, dict(iters=info.iters, true_relres=info.true_relres)

    def ip_prepare(self, f, params, st):
        rhs = self._empty(self.n_slots + 1)
        s = self._state_struct(st)
        self._call(self.lib.ipmg_ip_prepare, self._ptr(f, self.n_slots, "f"), C.byref(params), C.byref(s),
                   self._ptr(rhs, self.n_slots + 1, "rhs"))
        return rhs

    def ip_step(self, f, params, st, simp=None):
        """One Newton step; simp=(rmin, p): on the SIMP model (Sec. 9)."""
        s = self._state_struct(st)
        info = L.IPInfo()
        allow = (L.E_STALLED, L.E_BREAKDOWN, L.E_NOT_CONVERGED)
        if simp is None:
            rc = self._call(self.lib.ipmg_ip_step, self._ptr(f, self.n_slots, "f"), C.byref(params), C.byref(s),
                            C.byref(info), allow=allow)
        else:
            rc = self._call(self.lib.ipmg_simp_ip_step, self._ptr(f, self.n_slots, "f"), C.byref(params),
                            float(simp[0]), float(simp[1]), C.byref(s), C.byref(info), allow=allow)
        self._state_back(s, st)
        return dict(alpha=info.alpha, nwt=info.nwt, gap=info.gap, volume_res=info.volume_res,
                    compliance=info.compliance, pcg_iters=info.pcg_iters, pcg_status=info.pcg_status,
                    pcg_true_relres=info.pcg_true_relres, pcg_retries=info.pcg_retries,
                    barrier_updated=info.barrier_updated,
                    converged=info.converged, setup_ms=info.setup_ms, solve_ms=info.solve_ms, rc=rc)

    def ip_run(self, f, params, callback=None, cg_tol_factor=1.0, simp=None):
        """Interior-point loop (Sec. 3.1): init, then Newton steps until the stop rule.
        log["short_solves"] counts Newton systems whose solve stopped at pcg_maxit and
        was taken as an inexact direction (true residual within accept_rtol); a solve
        that broke down or stopped above that bound ends the run ("solve_failed").
        cg_tol_factor < 1: the "CG tol decreasing" variant of Sec. 8.1, the PCG
        tolerance multiplied by this factor after every barrier update (0.5 there).
        simp=(rmin, p): the SIMP model with the density filter (Sec. 9)."""
        params = L.IPParams.from_buffer_copy(params)
        st, init = self.ip_init(f, params, simp=simp)
        log = dict(newton=0, barrier_updates=0, pcg_iters=[init["iters"]], steps=[], status="max_newton",
                   short_solves=0, retries=0)
        while log["newton"] < params.max_newton:
            inf = self.ip_step(f, params, st, simp=simp)
            if inf["rc"] in (L.E_BREAKDOWN, L.E_NOT_CONVERGED):
                log["steps"].append(inf)
                log["status"] = "solve_failed"
                break
            log["newton"] += 1
            log["pcg_iters"].append(inf["pcg_iters"])
            log["steps"].append(inf)
            log["barrier_updates"] += inf["barrier_updated"]
            log["short_solves"] += int(inf["pcg_status"] != L.OK)
            log["retries"] += inf["pcg_retries"]
            if inf["barrier_updated"] and cg_tol_factor != 1.0:
                params.pcg_rtol *= cg_tol_factor
            if callback:
                callback(st, inf)
            if inf["rc"] == L.E_STALLED:
                log["status"] = "stalled"
                break
            if inf["converged"]:
                log["status"] = "converged"
                break
        return st, log
