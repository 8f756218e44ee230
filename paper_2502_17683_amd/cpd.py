"""Python face of the C-ABI: the ``CPD`` plan object and the kernel test hooks.

PyTorch supplies device memory (the workspace and the input/output
tensors) and the current HIP stream; nothing here computes.
"""
import ctypes

import torch

from . import _lib
from ._lib import CpdDesc, CpdStats, check, PRECISIONS


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _dev_f64(t, device):
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    return t.contiguous()


class CPD:
    """One CP-ALS run of the THC tensor (X[0..3], Z) at CP rank r_cp.

    X: one tensor (used for all four modes) or a list of four n_m x r_thc
    tensors; Z: r_thc x r_thc; init: four n_m x r_cp initial factors.
    Inputs are copied to the device as float64 if needed and kept alive by
    the object (the library borrows them).
    """

    def __init__(self, X, Z, r_cp, init, precision="fp64", tol=1e-4, fit_floor=1e-7,
                 chol_fallback=True, use_graph=True, fit_every=1, autotune=False, solve_panel=0,
                 device="cuda", tied=False, norm2=None, fit_target=0.0):
        """tied: the particle-tied model F1 = F0, F3 = F2 (symmetric ALS;
        FP64/FP32 only; init[1] and init[3] are not used).  norm2: optional
        one-element device tensor holding ||G||^2 (skips its O(R_thc^3)
        set-up; see df_to_thc)."""
        self.lib = _lib.load()
        self.device = torch.device(device)
        if not isinstance(X, (list, tuple)):
            X = [X] * 4
        xs, seen = [], {}
        for x in X:
            key = id(x)
            if key not in seen:
                seen[key] = _dev_f64(x, self.device)
            xs.append(seen[key])
        self.X = xs
        self.Z = _dev_f64(Z, self.device)
        self.init = [_dev_f64(f, self.device) for f in init]
        self.n = [int(x.shape[0]) for x in self.X]
        self.r_thc = int(self.Z.shape[0])
        self.r_cp = int(r_cp)
        d = CpdDesc()
        for m in range(4):
            d.n[m] = self.n[m]
            d.X[m] = self.X[m].data_ptr()
            d.init[m] = self.init[m].data_ptr()
        d.r_thc = self.r_thc
        d.r_cp = self.r_cp
        d.Z = self.Z.data_ptr()
        d.precision = PRECISIONS[precision]
        d.tol = float(tol)
        d.fit_floor = float(fit_floor)
        d.chol_fallback = int(bool(chol_fallback))
        d.use_graph = int(bool(use_graph))
        d.fit_every = int(fit_every)
        d.autotune = int(bool(autotune))
        d.solve_panel = int(solve_panel)
        d.tied = int(bool(tied))
        self.norm2 = None if norm2 is None else norm2.to(device=self.device, dtype=torch.float64).contiguous()
        d.norm2 = self.norm2.data_ptr() if self.norm2 is not None else None
        d.fit_target = float(fit_target)
        d.stream = _stream(self.device).value
        need = self.lib.cpd_workspace_size(ctypes.byref(d))
        if need == 0:
            raise _lib.CpdError(_lib.CPD_ERR_INVALID_ARG, "cpd_workspace_size")
        self.workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        d.workspace = self.workspace.data_ptr()
        d.workspace_bytes = need
        self.desc = d
        plan = ctypes.c_void_p()
        check(self.lib.cpd_init(ctypes.byref(d), ctypes.byref(plan)), "cpd_init")
        self.plan = plan

    @property
    def workspace_bytes(self):
        return self.desc.workspace_bytes

    def sweep(self, n=1, sync=True):
        """Run up to n sweeps; with sync, returns the list of fits (-1 for
        sweeps whose fit was not evaluated) and stops at convergence."""
        if not sync:
            check(self.lib.cpd_sweep(self.plan, int(n), None, None), "cpd_sweep")
            return None
        fits = (ctypes.c_double * max(int(n), 1))()
        ran = ctypes.c_int32(0)
        check(self.lib.cpd_sweep(self.plan, int(n), fits, ctypes.byref(ran)), "cpd_sweep")
        return list(fits[: ran.value])

    def run_logged(self, max_sweeps, path):
        """Run up to max_sweeps sweeps one at a time (each synchronised) and
        append one JSON line per sweep to `path`: sweep, fit (null where it
        was not evaluated), relative fit change, wall time of the sweep,
        damped-retry count, condition estimate of the last normal matrix,
        whether the problem runs on the FP64 products.  Stops at
        convergence.  Returns the list of fits."""
        import json
        import time
        fits, prev = [], None
        with open(path, "a") as out:
            for _ in range(int(max_sweeps)):
                t0 = time.perf_counter()
                got = self.sweep(1)
                dt = (time.perf_counter() - t0) * 1e3
                if not got:
                    break
                st = self.stats()
                f = got[0] if got[0] >= 0 else None
                rel = (abs(f - prev) / prev) if (f is not None and prev) else None
                out.write(json.dumps({"sweep": int(st["sweeps"]), "fit": f, "dfit_rel": rel, "t_sweep_ms": dt,
                                      "chol_fallbacks": int(st["fallbacks"]), "condV_est": float(st["cond_est"]),
                                      "fp64_path": int(st["fp64_path"])}) + "\n")
                fits.append(got[0])
                if f is not None:
                    prev = f
                if st["converged"]:
                    break
        return fits

    def fit(self):
        f = ctypes.c_double()
        check(self.lib.cpd_fit(self.plan, ctypes.byref(f)), "cpd_fit")
        return f.value

    def factors(self):
        F = [torch.empty(n, self.r_cp, dtype=torch.float64, device=self.device) for n in self.n]
        lam = torch.empty(self.r_cp, dtype=torch.float64, device=self.device)
        arr = (ctypes.c_void_p * 4)(*[f.data_ptr() for f in F])
        check(self.lib.cpd_get_factors(self.plan, arr, _ptr(lam)), "cpd_get_factors")
        torch.cuda.current_stream(self.device).synchronize()
        return F, lam

    def set_factors(self, F, lam, prev_fit=-1.0, sweeps=0):
        F = [_dev_f64(f, self.device) for f in F]
        lam = _dev_f64(lam, self.device)
        arr = (ctypes.c_void_p * 4)(*[f.data_ptr() for f in F])
        check(self.lib.cpd_set_factors(self.plan, arr, _ptr(lam), float(prev_fit), int(sweeps)),
              "cpd_set_factors")
        torch.cuda.current_stream(self.device).synchronize()

    def stats(self):
        s = CpdStats()
        check(self.lib.cpd_stats(self.plan, ctypes.byref(s)), "cpd_stats")
        return {k: getattr(s, k) for k, _ in CpdStats._fields_}

    def mttkrp(self, mode):
        M = torch.empty(self.n[mode], self.r_cp, dtype=torch.float64, device=self.device)
        check(self.lib.cpd_mttkrp(self.plan, int(mode), _ptr(M)), "cpd_mttkrp")
        torch.cuda.current_stream(self.device).synchronize()
        return M

    def autotune_log(self):
        """The autotuner's decisions for this plan ("kind,dims=shape" lines)."""
        n = self.lib.cpd_autotune_log(self.plan, None, 0)
        buf = ctypes.create_string_buffer(max(n, 0) + 1)
        self.lib.cpd_autotune_log(self.plan, buf, len(buf))
        return buf.value.decode()

    def kernel_times(self, reps=5):
        """Average ms of (projection, core product, back-projection, Gram,
        solve, V + factorisation + forward solve, backward solve, V) at this
        plan's shapes.  Invalidates the plan's state."""
        out = (ctypes.c_double * 8)()
        check(self.lib.cpd_kernel_times(self.plan, int(reps), out), "cpd_kernel_times")
        return dict(zip(("projection", "core", "backprojection", "gram", "solve", "factor_fwd",
                         "solve_bwd", "form_v"), list(out)))

    def close(self):
        if getattr(self, "plan", None) is not None and self.plan.value:
            self.lib.cpd_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CPDBatch:
    """Many independent CP-ALS problems of uneven size run as one grouped
    sweep (one launch per step for all problems, one hipGraph per sweep).

    problems: list of dicts with keys X (tensor or list of 4), Z, r_cp, init
    (list of 4).  Options are shared by all problems.
    """

    def __init__(self, problems, precision="mixed", tol=1e-4, fit_floor=1e-7, chol_fallback=True,
                 use_graph=True, fit_every=1, autotune=False, solve_panel=0, device="cuda", tied=False,
                 fit_targets=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.count = len(problems)
        self._keep = []
        descs = (CpdDesc * self.count)()
        self.shapes = []
        cache = {}

        def dev(t):
            key = id(t)
            if key not in cache:
                cache[key] = _dev_f64(t, self.device)
                self._keep.append(cache[key])
            return cache[key]

        for i, pr in enumerate(problems):
            X = pr["X"] if isinstance(pr["X"], (list, tuple)) else [pr["X"]] * 4
            Xs = [dev(x) for x in X]
            Zd = dev(pr["Z"])
            init = [_dev_f64(f, self.device) for f in pr["init"]]
            self._keep.extend(init)
            d = descs[i]
            for m in range(4):
                d.n[m] = int(Xs[m].shape[0])
                d.X[m] = Xs[m].data_ptr()
                d.init[m] = init[m].data_ptr()
            d.r_thc = int(Zd.shape[0])
            d.r_cp = int(pr["r_cp"])
            d.Z = Zd.data_ptr()
            d.precision = PRECISIONS[precision]
            d.tol = float(tol)
            d.fit_floor = float(fit_floor)
            d.chol_fallback = int(bool(chol_fallback))
            d.use_graph = int(bool(use_graph))
            d.fit_every = int(fit_every)
            d.autotune = int(bool(autotune))
            d.solve_panel = int(solve_panel)
            d.tied = int(bool(tied))
            d.fit_target = float(fit_targets[i]) if fit_targets is not None else 0.0
            d.stream = _stream(self.device).value
            self.shapes.append(([d.n[m] for m in range(4)], d.r_thc, d.r_cp))
        need = self.lib.cpd_batch_workspace_size(descs, self.count)
        if need == 0:
            raise _lib.CpdError(_lib.CPD_ERR_INVALID_ARG, "cpd_batch_workspace_size")
        self.workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        self.descs = descs
        plan = ctypes.c_void_p()
        check(self.lib.cpd_batch_init(descs, self.count, ctypes.c_void_p(self.workspace.data_ptr()), need,
                                      ctypes.byref(plan)), "cpd_batch_init")
        self.plan = plan

    def sweep(self, n=1, sync=True):
        """Run up to n batched sweeps.  With sync, returns one list of fits
        per problem, covering the sweeps that problem actually ran (-1 where
        the fit was not evaluated)."""
        if not sync:
            check(self.lib.cpd_batch_sweep(self.plan, int(n), None, None), "cpd_batch_sweep")
            return None
        _, _, before = self.states()
        fits = (ctypes.c_double * (self.count * max(int(n), 1)))()
        ran = ctypes.c_int32(0)
        check(self.lib.cpd_batch_sweep(self.plan, int(n), fits, ctypes.byref(ran)), "cpd_batch_sweep")
        _, _, after = self.states()
        return [list(fits[i * n: i * n + min(ran.value, after[i] - before[i])]) for i in range(self.count)]

    def states(self):
        f = (ctypes.c_double * self.count)()
        c = (ctypes.c_int32 * self.count)()
        s = (ctypes.c_int32 * self.count)()
        check(self.lib.cpd_batch_states(self.plan, f, c, s), "cpd_batch_states")
        return list(f), list(c), list(s)

    def factors(self, idx):
        n, _, r_cp = self.shapes[idx]
        F = [torch.empty(k, r_cp, dtype=torch.float64, device=self.device) for k in n]
        lam = torch.empty(r_cp, dtype=torch.float64, device=self.device)
        arr = (ctypes.c_void_p * 4)(*[f.data_ptr() for f in F])
        check(self.lib.cpd_batch_get_factors(self.plan, int(idx), arr, _ptr(lam)), "cpd_batch_get_factors")
        torch.cuda.current_stream(self.device).synchronize()
        return F, lam

    def stats(self, idx):
        st = CpdStats()
        check(self.lib.cpd_batch_stats(self.plan, int(idx), ctypes.byref(st)), "cpd_batch_stats")
        return {k: getattr(st, k) for k, _ in CpdStats._fields_}

    def kernel_times(self, reps=5):
        out = (ctypes.c_double * 8)()
        check(self.lib.cpd_kernel_times(self.plan, int(reps), out), "cpd_kernel_times")
        return dict(zip(("projection", "core", "backprojection", "gram", "solve", "factor_fwd",
                         "solve_bwd", "form_v"), list(out)))

    def autotune_log(self):
        n = self.lib.cpd_autotune_log(self.plan, None, 0)
        buf = ctypes.create_string_buffer(max(n, 0) + 1)
        self.lib.cpd_autotune_log(self.plan, buf, len(buf))
        return buf.value.decode()

    def close(self):
        if getattr(self, "plan", None) is not None and self.plan.value:
            self.lib.cpd_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lt_scale_rows(X, eps, t, sign):
    """exp(sign * eps_p * t) * X[p, :] on the GPU (Laplace-transform row scaling)."""
    lib = _lib.load()
    X = X.contiguous()
    eps = eps.contiguous()
    out = torch.empty_like(X)
    check(lib.cpd_lt_scale_rows(_ptr(X), _ptr(eps), X.shape[0], X.shape[1], float(t), float(sign), _ptr(out),
                                _stream(X.device)), "cpd_lt_scale_rows")
    return out


def test_gemm(A, B1, B2=None, a_t=False, b_t=False):
    """C = op(A) op(B1 [o B2]) through the library's FP64/FP32 GEMM."""
    lib = _lib.load()
    fp32 = A.dtype == torch.float32
    M = A.shape[1] if a_t else A.shape[0]
    K = A.shape[0] if a_t else A.shape[1]
    N = B1.shape[0] if b_t else B1.shape[1]
    C = torch.empty(M, N, dtype=A.dtype, device=A.device)
    check(lib.cpd_test_gemm(int(fp32), M, N, K, _ptr(A), A.shape[1], int(a_t), _ptr(B1), _ptr(B2),
                            B1.shape[1], int(b_t), _ptr(C), N, _stream(A.device)), "cpd_test_gemm")
    torch.cuda.current_stream(A.device).synchronize()
    return C


def test_flow_spin_limit(polls):
    """Polls a dataflow-solve wait makes before giving up (negative: the
    default); returns the previous value.  Failure-path tests only."""
    return int(_lib.load().cpd_test_flow_spin_limit(int(polls)))


def test_bwd_form(form):
    """Form of the one-level backward solve of plans and test solves
    created afterwards: 0 (default) two block columns per dependency hop,
    1 one per hop; returns the previous form."""
    return int(_lib.load().cpd_test_bwd_form(int(form)))


def test_split_force(code):
    """Forces the split-BF16 launch shape of plans created afterwards (the
    cpd_autotune_log shape code; 0: off); returns the previous code."""
    return int(_lib.load().cpd_test_split_force(int(code)))


def test_solve(V, M, panel=0):
    """F = M V^{-1} through the library's blocked Cholesky and solves
    (panels of `panel` 64-wide blocks; 0: one level)."""
    lib = _lib.load()
    fp32 = V.dtype == torch.float32
    R, n = V.shape[0], M.shape[0]
    ws = torch.empty(lib.cpd_test_solve_workspace(int(fp32), R, n), dtype=torch.uint8, device=V.device)
    F = torch.empty_like(M)
    failed = ctypes.c_int32(0)
    code = lib.cpd_test_solve(int(fp32), R, n, _ptr(V), _ptr(M), _ptr(F), _ptr(ws), ws.numel(),
                              _stream(V.device), ctypes.byref(failed), int(panel))
    if code not in (_lib.CPD_OK, _lib.CPD_ERR_NOT_SPD):
        check(code, "cpd_test_solve")
    return F, bool(failed.value)


def test_gemm_split(A, B, A2=None, bm=0, B2=None, wide=False, kparts=1):
    """C = A B^T through the split-BF16 GEMM, with A (B) replaced by the
    FP32 product A o A2 (B o B2) when given.  Launch shape: 128-column tiles
    with bm = 64 or 128 rows (0: the sweep's heuristic), with wide=True
    bm x 256 tiles (bm = 128 or 256) and kparts K slices, or with wide=2
    256 x 256 direct-load tiles of pre-split operands and kparts K slices."""
    lib = _lib.load()
    M, K = A.shape
    N = B.shape[0]
    ws = torch.empty(lib.cpd_test_split_workspace(M, N, K), dtype=torch.uint8, device=A.device)
    C = torch.empty(M, N, dtype=torch.float64, device=A.device)
    check(lib.cpd_test_gemm_split(M, N, K, _ptr(A), _ptr(A2), _ptr(B), _ptr(B2), _ptr(C), _ptr(ws), ws.numel(),
                                  _stream(A.device), int(bm), 2 if wide == 2 else int(bool(wide)), int(kparts)),
          "cpd_test_gemm_split")
    torch.cuda.current_stream(A.device).synchronize()
    return C


def df_to_thc(B, n):
    """The exact THC form (X0, X1, Z, norm2) of the DF tensor
    G[p,q,r,s] = sum_X B[(p,q),X] B[(r,s),X] (eq. df_loss) on the GPU: pair
    selection factors, Z = B B^T and ||G||^2 = ||B^T B||_F^2 (one-element
    tensor); CPD([X0, X1, X0, X1], Z, ..., norm2=norm2) then runs the
    CP-ALS of the DF loss."""
    lib = _lib.load()
    B = B.contiguous()
    nn = n * n
    X0 = torch.empty(n, nn, dtype=torch.float64, device=B.device)
    X1 = torch.empty(n, nn, dtype=torch.float64, device=B.device)
    Z = torch.empty(nn, nn, dtype=torch.float64, device=B.device)
    norm2 = torch.empty(1, dtype=torch.float64, device=B.device)
    check(lib.cpd_df_to_thc(int(n), int(B.shape[1]), _ptr(B), _ptr(X0), _ptr(X1), _ptr(Z), _ptr(norm2),
                            _stream(B.device)), "cpd_df_to_thc")
    return X0, X1, Z, norm2
