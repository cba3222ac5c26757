"""ctypes binding of librpca (``include/rpca.h``): argument marshalling only.

Every function has the name and argument order of the C entry point.  Device
buffers are torch tensors on the context's device (used only as device memory
and for their streams); layouts are column-major, so an m x n matrix with
leading dimension ld is a row-major torch tensor of shape (n, ld).  Negative
statuses raise :class:`RpcaError`; positive statuses (warnings) are returned.

There is no fallback: if ``librpca.so`` has not been built, importing this
module raises.
"""
from __future__ import annotations

import ctypes
import pathlib

import numpy as np

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "librpca.so"
if not _LIB_PATH.exists():
    raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() or "
                      "python paper_1108_5359_amd/build.py")
lib = ctypes.CDLL(str(_LIB_PATH))

RPCA_OK = 0
RPCA_WARN_NOT_CONVERGED = 1
RPCA_WARN_RANK = 2
RPCA_ERR_ARG = -1
RPCA_ERR_NOMEM = -2
RPCA_ERR_DEVICE = -3
RPCA_ERR_SEED = -4
RPCA_ERR_NUMERIC = -5
RPCA_SEED_ROUTE_EIGEN = 1
RPCA_SEED_ROUTE_SUBSPACE = 2
RPCA_SEED_ROUTE_LDS_JACOBI = 3
RPCA_SEED_ROUTE_FELL_BACK = 4
RPCA_ERR_UNSUPPORTED = -6
RPCA_ITERS_BAD_INDEX = -2147483648
RPCA_ITERS_NONFINITE = -2147483647


class rpca_opts(ctypes.Structure):
    _fields_ = [
        ("os_r", ctypes.c_int32), ("os_c", ctypes.c_int32),
        ("seed_lambda", ctypes.c_double), ("seed_tol", ctypes.c_double),
        ("seed_rho", ctypes.c_double), ("seed_mu0_scale", ctypes.c_double),
        ("seed_mu_max_scale", ctypes.c_double), ("seed_max_iter", ctypes.c_int32),
        ("seed_rank_floor", ctypes.c_double),
        ("filt_eps", ctypes.c_double), ("filt_rho", ctypes.c_double),
        ("filt_beta0_scale", ctypes.c_double), ("filt_beta_max_scale", ctypes.c_double),
        ("filt_max_iter", ctypes.c_int32), ("filt_refresh", ctypes.c_int32),
        ("rng_seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
        ("overlap_chunks", ctypes.c_int32), ("filter_form", ctypes.c_int32),
        ("seed_route", ctypes.c_int32),
    ]


class rpca_info(ctypes.Structure):
    _fields_ = [
        ("r_used", ctypes.c_int32), ("seed_iters", ctypes.c_int32),
        ("seed_converged", ctypes.c_int32), ("filt_iters_max", ctypes.c_int32),
        ("filt_iters_total", ctypes.c_int64), ("filt_not_converged", ctypes.c_int64),
        ("t_seed_ms", ctypes.c_double), ("t_filter_ms", ctypes.c_double),
        ("t_reconstruct_ms", ctypes.c_double), ("seed_route", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32

lib.rpca_opts_default.argtypes = [ctypes.POINTER(rpca_opts)]
lib.rpca_opts_default.restype = None
lib.rpca_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(_vp)]
lib.rpca_ctx_destroy.argtypes = [_vp]
lib.rpca_last_error.argtypes = [_vp]
lib.rpca_last_error.restype = ctypes.c_char_p
lib.rpca_status_string.argtypes = [ctypes.c_int]
lib.rpca_status_string.restype = ctypes.c_char_p
lib.rpca_sample_indices.argtypes = [_i64, _i64, _i64, _i64, ctypes.c_uint64, _vp, _vp]
lib.rpca_filter_form.argtypes = [_vp, _i64, _i32, _i64, ctypes.POINTER(rpca_opts), ctypes.POINTER(_i32)]
lib.rpca_last_seed_route.argtypes = [_vp, ctypes.POINTER(_i32)]
lib.rpca_seed.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _i32,
                          ctypes.POINTER(rpca_opts), _vp, _vp, _vp,
                          ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
lib.rpca_filter_cols.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i32,
                                 ctypes.POINTER(rpca_opts), _vp, _vp, _vp]
lib.rpca_filter_rows.argtypes = lib.rpca_filter_cols.argtypes
lib.rpca_filter.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                            _vp, _vp, _i32, ctypes.POINTER(rpca_opts), _vp, _vp, _vp, _vp, _vp]
lib.rpca_reconstruct.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp,
                                 _vp, _i32, _vp, _vp, _vp, _i64, _vp, _i64, _vp]
lib.rpca_reconstruct_noalloc.argtypes = lib.rpca_reconstruct.argtypes
lib.rpca_reconstruct_noalloc.restype = ctypes.c_int
RPCA_NOALLOC_SCRATCH_BYTES = 32 << 20
lib.rpca_filter_complete.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp,
                                     _vp, _vp, _vp, _i32, ctypes.POINTER(rpca_opts), _vp, _vp,
                                     _vp, _vp, _vp, _i64, _vp, _i64, _vp]
lib.rpca_filter_complete.restype = ctypes.c_int
lib.rpca_solve.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, ctypes.POINTER(rpca_opts), _vp,
                           _vp, _vp, _i64, _vp, _i64, ctypes.POINTER(rpca_info), _vp]
for _f in ("rpca_ctx_create", "rpca_ctx_destroy", "rpca_sample_indices", "rpca_seed",
           "rpca_filter", "rpca_filter_cols", "rpca_filter_rows", "rpca_reconstruct", "rpca_solve"):
    getattr(lib, _f).restype = ctypes.c_int


class RpcaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{rpca_status_string(status)}: {message}")
        self.status = status


def rpca_status_string(status: int) -> str:
    return lib.rpca_status_string(int(status)).decode()


def rpca_opts_default(**overrides) -> rpca_opts:
    o = rpca_opts()
    lib.rpca_opts_default(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class Context:
    """Owns an ``rpca_ctx_t`` on one device."""

    def __init__(self, device: int = 0):
        h = _vp()
        st = lib.rpca_ctx_create(int(device), ctypes.byref(h))
        if st != RPCA_OK:
            raise RpcaError(st, lib.rpca_last_error(None).decode())
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib.rpca_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int) -> int:
        if st < 0:
            raise RpcaError(st, lib.rpca_last_error(self.handle).decode())
        return st

    def last_error(self) -> str:
        return lib.rpca_last_error(self.handle).decode()


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def rpca_sample_indices(m: int, n: int, p: int, q: int, seed: int):
    rows = np.empty(p, dtype=np.int64)
    cols = np.empty(q, dtype=np.int64)
    st = lib.rpca_sample_indices(m, n, p, q, ctypes.c_uint64(seed), rows.ctypes.data, cols.ctypes.data)
    if st != RPCA_OK:
        raise RpcaError(st, "invalid sampling sizes")
    return rows, cols


def rpca_seed(ctx: Context, M, m, n, ldm, seed_rows, p, seed_cols, q, r, opts, U, sigma, V):
    ru = _i32(0)
    it = _i32(0)
    st = ctx.check(lib.rpca_seed(ctx.handle, _ptr(M), m, n, ldm, _ptr(seed_rows), p,
                                 _ptr(seed_cols), q, r, ctypes.byref(opts), _ptr(U), _ptr(sigma),
                                 _ptr(V), ctypes.byref(ru), ctypes.byref(it)))
    return st, ru.value, it.value


def rpca_last_seed_route(ctx: Context) -> int:
    """Route the last rpca_seed call on ctx took (RPCA_SEED_ROUTE_*)."""
    route = _i32(0)
    ctx.check(lib.rpca_last_seed_route(ctx.handle, ctypes.byref(route)))
    return route.value


def rpca_filter_form(ctx: Context, p: int, r: int, nreg: int, opts) -> int:
    """The filter kernel form a call takes: 0 FP16 precision form, 1 FP32 tile, 2 FP32 split."""
    f = _i32(0)
    ctx.check(lib.rpca_filter_form(ctx.handle, p, r, nreg, ctypes.byref(opts), ctypes.byref(f)))
    return f.value


def rpca_filter_cols(ctx: Context, M, m, n, ldm, seed_rows, p, cols, nc, U, r, opts, Qt, iters,
                     stream=None):
    return ctx.check(lib.rpca_filter_cols(ctx.handle, _ptr(M), m, n, ldm, _ptr(seed_rows), p,
                                          _ptr(cols), nc, _ptr(U), r, ctypes.byref(opts), _ptr(Qt),
                                          _ptr(iters), _stream(stream)))


def rpca_filter_rows(ctx: Context, M, m, n, ldm, seed_cols, q, rows, nr, V, r, opts, Pt, iters,
                     stream=None):
    return ctx.check(lib.rpca_filter_rows(ctx.handle, _ptr(M), m, n, ldm, _ptr(seed_cols), q,
                                          _ptr(rows), nr, _ptr(V), r, ctypes.byref(opts), _ptr(Pt),
                                          _ptr(iters), _stream(stream)))


def rpca_filter(ctx: Context, M, m, n, ldm, seed_rows, p, seed_cols, q, cols, nc, rows, nr, U, V,
                r, opts, Qt, col_iters, Pt, row_iters, stream=None):
    return ctx.check(lib.rpca_filter(ctx.handle, _ptr(M), m, n, ldm, _ptr(seed_rows), p,
                                     _ptr(seed_cols), q, _ptr(cols), nc, _ptr(rows), nr, _ptr(U),
                                     _ptr(V), r, ctypes.byref(opts), _ptr(Qt), _ptr(col_iters),
                                     _ptr(Pt), _ptr(row_iters), _stream(stream)))


def rpca_reconstruct(ctx: Context, M, m, n, ldm, seed_rows, p, seed_cols, q, U, sigma, V, r, Qt,
                     Pt, L, ldl, S, lds, stream=None):
    return ctx.check(lib.rpca_reconstruct(ctx.handle, _ptr(M), m, n, ldm, _ptr(seed_rows), p,
                                          _ptr(seed_cols), q, _ptr(U), _ptr(sigma), _ptr(V), r,
                                          _ptr(Qt), _ptr(Pt), _ptr(L), ldl, _ptr(S), lds,
                                          _stream(stream)))


def rpca_reconstruct_noalloc(ctx: Context, M, m, n, ldm, seed_rows, p, seed_cols, q, U, sigma, V,
                             r, Qt, Pt, L, ldl, S, lds, stream=None):
    return ctx.check(lib.rpca_reconstruct_noalloc(ctx.handle, _ptr(M), m, n, ldm, _ptr(seed_rows), p,
                                                  _ptr(seed_cols), q, _ptr(U), _ptr(sigma), _ptr(V),
                                                  r, _ptr(Qt), _ptr(Pt), _ptr(L), ldl, _ptr(S), lds,
                                                  _stream(stream)))


def rpca_solve(ctx: Context, M, m, n, ldm, r, opts, seed_rows, seed_cols, L, ldl, S, lds,
               stream=None):
    info = rpca_info()
    st = ctx.check(lib.rpca_solve(ctx.handle, _ptr(M), m, n, ldm, r, ctypes.byref(opts),
                                  _ptr(seed_rows), _ptr(seed_cols), _ptr(L), ldl, _ptr(S), lds,
                                  ctypes.byref(info), _stream(stream)))
    return st, info


# ---------------------------------------------------------------- batched form
class rpca_job(ctypes.Structure):
    _fields_ = [
        ("M", _vp), ("m", _i64), ("n", _i64), ("ldm", _i64), ("r", _i32),
        ("seed_rows", _vp), ("p", _i64), ("seed_cols", _vp), ("q", _i64),
        ("L", _vp), ("ldl", _i64), ("S", _vp), ("lds", _i64),
    ]


class rpca_batch_tuning(ctypes.Structure):
    _fields_ = [
        ("lane_max_p", _i32), ("lane_max_r", _i32), ("lane_split2_p", _i32),
        ("lane_split4_p", _i32), ("filter_waves_per_cu", _i32),
        ("recon_cols_per_wave", _i32), ("order", _i32), ("graph", _i32), ("seed_batched", _i32),
        ("recon_waves_per_cu", _i32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


lib.rpca_batch_tuning_default.argtypes = [ctypes.POINTER(rpca_batch_tuning)]
lib.rpca_batch_tuning_default.restype = None
lib.rpca_batch_create.argtypes = [_vp, ctypes.POINTER(rpca_job), _i64, ctypes.POINTER(rpca_opts),
                                  ctypes.POINTER(rpca_batch_tuning), ctypes.POINTER(_vp)]
lib.rpca_batch_seed.argtypes = [_vp, _vp]
lib.rpca_batch_run.argtypes = [_vp, _vp]
lib.rpca_batch_job_info.argtypes = [_vp, _i64, ctypes.POINTER(rpca_info)]
lib.rpca_batch_destroy.argtypes = [_vp]
lib.rpca_batch_job_factors.argtypes = [_vp, _i64, _vp, _vp, _vp]
for _f in ("rpca_batch_create", "rpca_batch_seed", "rpca_batch_run", "rpca_batch_job_info",
           "rpca_batch_destroy", "rpca_batch_job_factors"):
    getattr(lib, _f).restype = ctypes.c_int


def rpca_batch_tuning_default(**overrides) -> rpca_batch_tuning:
    t = rpca_batch_tuning()
    lib.rpca_batch_tuning_default(ctypes.byref(t))
    for k, v in overrides.items():
        if not hasattr(t, k):
            raise AttributeError(k)
        setattr(t, k, v)
    return t


def job(M, m, n, ldm, r, seed_rows, p, seed_cols, q, L, ldl, S, lds) -> rpca_job:
    """One ``rpca_job`` from device tensors (kept alive by the caller)."""
    return rpca_job(_ptr(M), m, n, ldm, r, _ptr(seed_rows), p, _ptr(seed_cols), q, _ptr(L), ldl,
                    _ptr(S), lds)


class Batch:
    """Owns an ``rpca_batch_t``; errors are reported on the owner context."""

    def __init__(self, ctx: Context, jobs, opts, tuning=None):
        arr = (rpca_job * len(jobs))(*jobs)
        h = _vp()
        ctx.check(lib.rpca_batch_create(ctx.handle, arr, len(jobs), ctypes.byref(opts),
                                        ctypes.byref(tuning) if tuning is not None else None,
                                        ctypes.byref(h)))
        self.ctx = ctx
        self.handle = h
        self.njobs = len(jobs)

    def close(self):
        if self.handle:
            lib.rpca_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rpca_batch_create(ctx: Context, jobs, opts, tuning=None) -> Batch:
    return Batch(ctx, jobs, opts, tuning)


def rpca_batch_seed(batch: Batch, stream=None) -> int:
    return batch.ctx.check(lib.rpca_batch_seed(batch.handle, _stream(stream)))


def rpca_batch_run(batch: Batch, stream=None) -> int:
    return batch.ctx.check(lib.rpca_batch_run(batch.handle, _stream(stream)))


def rpca_batch_job_info(batch: Batch, job_index: int):
    info = rpca_info()
    st = batch.ctx.check(lib.rpca_batch_job_info(batch.handle, job_index, ctypes.byref(info)))
    return st, info


def rpca_batch_destroy(batch: Batch) -> None:
    batch.close()


def rpca_batch_job_factors(batch: Batch, job_index: int, U, sigma, V) -> int:
    """U: (r, p) FP64 tensor (column-major p x r), sigma: (r,), V: (r, q)."""
    return batch.ctx.check(lib.rpca_batch_job_factors(batch.handle, job_index, _ptr(U), _ptr(sigma),
                                                      _ptr(V)))


# ---------------------------------------------------------------- served form
class rpca_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_double), ("workers", _i32), ("max_batch", _i32)]


class rpca_request_info(ctypes.Structure):
    _fields_ = [("status", _i32), ("batch_size", _i32), ("info", rpca_info),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double)]


class rpca_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("failed", _i64), ("batches", _i64),
                ("queued", _i64), ("peak_inflight_bytes", ctypes.c_double),
                ("inflight_bytes", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


lib.rpca_server_opts_default.argtypes = [ctypes.POINTER(rpca_server_opts)]
lib.rpca_server_opts_default.restype = None
lib.rpca_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(rpca_opts),
                                   ctypes.POINTER(rpca_batch_tuning),
                                   ctypes.POINTER(rpca_server_opts), ctypes.POINTER(_vp)]
lib.rpca_server_submit.argtypes = [_vp, ctypes.POINTER(rpca_job), ctypes.POINTER(_i64)]
lib.rpca_server_wait.argtypes = [_vp, _i64, ctypes.POINTER(rpca_request_info)]
lib.rpca_server_poll.argtypes = [_vp, _i64, ctypes.POINTER(_i32)]
lib.rpca_server_get_stats.argtypes = [_vp, ctypes.POINTER(rpca_server_stats)]
lib.rpca_server_error.argtypes = [_vp]
lib.rpca_server_error.restype = ctypes.c_char_p
lib.rpca_server_destroy.argtypes = [_vp]
for _f in ("rpca_server_create", "rpca_server_submit", "rpca_server_wait", "rpca_server_poll",
           "rpca_server_get_stats", "rpca_server_destroy"):
    getattr(lib, _f).restype = ctypes.c_int


def rpca_server_opts_default(**overrides) -> rpca_server_opts:
    o = rpca_server_opts()
    lib.rpca_server_opts_default(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class Server:
    """Owns an ``rpca_server_t``: submit() queues a job, wait() returns its
    ``rpca_request_info`` (raising RpcaError for a failed request)."""

    def __init__(self, opts, tuning=None, server_opts=None, device: int = 0):
        h = _vp()
        st = lib.rpca_server_create(device, ctypes.byref(opts),
                                    ctypes.byref(tuning) if tuning is not None else None,
                                    ctypes.byref(server_opts) if server_opts is not None else None,
                                    ctypes.byref(h))
        if st != RPCA_OK:
            raise RpcaError(st, lib.rpca_server_error(None).decode())
        self.handle = h

    def submit(self, job: rpca_job) -> int:
        t = _i64(0)
        st = lib.rpca_server_submit(self.handle, ctypes.byref(job), ctypes.byref(t))
        if st != RPCA_OK:
            raise RpcaError(st, lib.rpca_server_error(self.handle).decode())
        return t.value

    def wait(self, ticket: int, check: bool = True) -> rpca_request_info:
        info = rpca_request_info()
        st = lib.rpca_server_wait(self.handle, ticket, ctypes.byref(info))
        if st < 0 and check:
            raise RpcaError(st, f"request {ticket} failed")
        return info

    def poll(self, ticket: int) -> bool:
        d = _i32(0)
        st = lib.rpca_server_poll(self.handle, ticket, ctypes.byref(d))
        if st != RPCA_OK:
            raise RpcaError(st, lib.rpca_server_error(self.handle).decode())
        return bool(d.value)

    def stats(self) -> rpca_server_stats:
        s = rpca_server_stats()
        lib.rpca_server_get_stats(self.handle, ctypes.byref(s))
        return s

    def close(self):
        if self.handle:
            lib.rpca_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rpca_filter_complete(ctx: Context, M, m, n, ldm, seed_rows, p, seed_cols, q, cols, rows, U, sigma,
                         V, r, opts, Qt, col_iters, Pt, row_iters, L, ldl, S, lds, stream=None):
    return ctx.check(lib.rpca_filter_complete(ctx.handle, _ptr(M), m, n, ldm, _ptr(seed_rows), p,
                                              _ptr(seed_cols), q, _ptr(cols), _ptr(rows), _ptr(U),
                                              _ptr(sigma), _ptr(V), r, ctypes.byref(opts), _ptr(Qt),
                                              _ptr(col_iters), _ptr(Pt), _ptr(row_iters), _ptr(L),
                                              ldl, _ptr(S), lds, _stream(stream)))


# ---------------------------------------------------------------- factored output, new columns
lib.rpca_solve_factored.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, ctypes.POINTER(rpca_opts),
                                    _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                    ctypes.POINTER(rpca_info), _vp]
lib.rpca_solve_factored.restype = ctypes.c_int
lib.rpca_filter_new_cols.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _vp, _i32, _vp,
                                     ctypes.POINTER(rpca_opts), _vp, _vp, _vp, _i64, _vp, _i64, _vp]
lib.rpca_filter_new_cols.restype = ctypes.c_int


def rpca_solve_factored(ctx: Context, M, m, n, ldm, r, opts, seed_rows, p, seed_cols, q, U, sigma,
                        V, Qt, col_iters, Pt, row_iters, stream=None):
    """Returns (status, rpca_info); Qt / Pt hold r_used rows (ld r_used)."""
    info = rpca_info()
    st = ctx.check(lib.rpca_solve_factored(ctx.handle, _ptr(M), m, n, ldm, r, ctypes.byref(opts),
                                           _ptr(seed_rows), p, _ptr(seed_cols), q, _ptr(U),
                                           _ptr(sigma), _ptr(V), _ptr(Qt), _ptr(col_iters), _ptr(Pt),
                                           _ptr(row_iters), ctypes.byref(info), _stream(stream)))
    return st, info


def rpca_filter_new_cols(ctx: Context, Mnew, m, nnew, ldm, seed_rows, p, U, sigma, r, Pt, opts,
                         Qt_new, iters, L, ldl, S, lds, stream=None):
    return ctx.check(lib.rpca_filter_new_cols(ctx.handle, _ptr(Mnew), m, nnew, ldm, _ptr(seed_rows),
                                              p, _ptr(U), _ptr(sigma), r, _ptr(Pt),
                                              ctypes.byref(opts), _ptr(Qt_new), _ptr(iters), _ptr(L),
                                              ldl, _ptr(S), lds, _stream(stream)))


# ---------------------------------------------------------------- target-rank estimation
RPCA_RANK_MAX_ROUNDS = 16


class rpca_rank_info(ctypes.Structure):
    _fields_ = [("r_est", _i32), ("accepted", _i32), ("rounds", _i32), ("cv_rank", _i32),
                ("p", _i64), ("q", _i64), ("ranks", _i32 * RPCA_RANK_MAX_ROUNDS),
                ("ps", _i64 * RPCA_RANK_MAX_ROUNDS), ("qs", _i64 * RPCA_RANK_MAX_ROUNDS)]


lib.rpca_estimate_rank.argtypes = [_vp, _vp, _i64, _i64, _i64, _i32, ctypes.POINTER(rpca_opts),
                                   _vp, _vp, _i32, ctypes.POINTER(rpca_rank_info)]
lib.rpca_estimate_rank.restype = ctypes.c_int


def rpca_estimate_rank(ctx: Context, M, m, n, ldm, r0, opts, row_order, col_order,
                       cross_validate=True):
    """row_order / col_order: host permutations (int64 numpy).  Returns
    (status, rpca_rank_info)."""
    ro = np.ascontiguousarray(row_order, dtype=np.int64)
    co = np.ascontiguousarray(col_order, dtype=np.int64)
    info = rpca_rank_info()
    st = ctx.check(lib.rpca_estimate_rank(ctx.handle, _ptr(M), m, n, ldm, r0, ctypes.byref(opts),
                                          ro.ctypes.data, co.ctypes.data, int(bool(cross_validate)),
                                          ctypes.byref(info)))
    return st, info
