"""Python binding of libshgb (ctypes): argument marshalling only.

Every step of the method runs in the HIP kernels behind the C ABI declared in
include/shgb.h; this module allocates device memory with torch, passes raw
pointers and the current HIP stream, and turns error codes into exceptions.
There is no CPU fallback: importing it without the built library raises.

The function names follow the C entry points: ``init_beams``,
``step_ensemble``, ``hop``, ``populations``, ``reconstruct``.
"""

import ctypes
import os

import torch  # loaded first: the library binds to the HIP runtime torch already holds

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshgb.so")

SHGB_OK = 0
SHGB_NCOMP = 4
SHGB_MAX_D = 12
SHGB_HOP_CAP = 16
SHGB_NDIAG = 8
SHGB_SCALAR_FIELDS = 8
PRECISION = {"fp64": 0, "mixed": 1}
DIST = {"normal": 0, "uniform": 1}
SHGB_SCHEME_RK4, SHGB_SCHEME_RK3 = 4, 3
SHGB_FIELD_DEFAULT, SHGB_FIELD_FP32_MATRIX = 0, 1
DIAG_NAMES = ("hops", "thr_ties", "dest_ties", "cap_overflow", "nonfinite", "nonspd",
              "zero_rate", "bad_index")


class ShgbError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {code} ({_lib.shgb_strerror(code).decode()})")
        self.code = code


_NC = SHGB_NCOMP


class LinQuad(ctypes.Structure):
    _fields_ = [("n_comp", ctypes.c_int32), ("a", (ctypes.c_double * 2) * _NC),
                ("J", ((ctypes.c_double * 2) * 2) * _NC), ("b0", ctypes.c_double * _NC),
                ("b", (ctypes.c_double * 2) * _NC), ("H", ((ctypes.c_double * 2) * 2) * _NC),
                ("gamma_re", (ctypes.c_double * _NC) * _NC), ("gamma_im", (ctypes.c_double * _NC) * _NC)]


class Model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("d", ctypes.c_int32), ("mass", ctypes.c_double),
                ("eps", ctypes.c_double), ("A", ctypes.c_double), ("B", ctypes.c_double),
                ("C", ctypes.c_double), ("D", ctypes.c_double), ("lam", ctypes.c_double),
                ("bath_omega", ctypes.c_double * (SHGB_MAX_D - 1)), ("lq", LinQuad)]


class StateDesc(ctypes.Structure):
    _fields_ = [("f64", ctypes.c_void_p), ("comp", ctypes.c_void_p), ("nhop", ctypes.c_void_p),
                ("n_beams", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("beam_id_offset", ctypes.c_uint64), ("m", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("f32", ctypes.c_void_p)]


class InitSpec(ctypes.Structure):
    _fields_ = [("q_mean", ctypes.c_double), ("q_std", ctypes.c_double), ("p_dist", ctypes.c_int32),
                ("p_a", ctypes.c_double), ("p_b", ctypes.c_double), ("comp0", ctypes.c_int32),
                ("a0", ctypes.c_double)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("tiles_per_grab", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class BatchDesc(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("d", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("total_tiles", ctypes.c_int64), ("cfg", BatchConfig),
                ("table", ctypes.c_void_p)]


SHGB_BATCH_WORK_BYTES = 256


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(python -m paper_1703_06116_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, V, I64, I32, U64, D = (ctypes.POINTER, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_uint64, ctypes.c_double)
    sig = {
        "shgb_init_beams": (I32, [P(Model), P(InitSpec), P(StateDesc), U64, V]),
        "shgb_step_ensemble": (I32, [P(Model), P(StateDesc), I32, D, U64, V, V]),
        "shgb_hop": (I32, [P(Model), P(StateDesc), V, I64, U64, V, V]),
        "shgb_step_ensemble_scheme": (I32, [P(Model), P(StateDesc), I32, D, U64, I32, V, V]),
        "shgb_populations_workspace": (I64, [I64, I32]),
        "shgb_populations": (I32, [P(Model), P(StateDesc), V, V, I64, V, V]),
        "shgb_populations_noalloc": (I32, [P(Model), P(StateDesc), V, V, V]),
        "shgb_population_stats": (I32, [V, I64, V, V]),
        "shgb_reconstruct_workspace": (I64, [I64, I32, I64]),
        "shgb_reconstruct": (I32, [P(Model), P(StateDesc), V, I64, V, V, I64, V]),
        "shgb_reconstruct_workspace_mode": (I64, [I64, I32, I64, I32]),
        "shgb_reconstruct_mode": (I32, [P(Model), P(StateDesc), V, I64, V, V, I64, I32, V]),
        "shgb_philox": (I32, [U64, V, V, I64, V]),
        "shgb_strerror": (ctypes.c_char_p, [I32]),
        "shgb_version": (I32, []),
        "shgb_abi_sizes": (None, [V]),
        "shgb_population_tangent_workspace": (I64, [I64]),
        "shgb_population_tangent": (I32, [P(Model), P(StateDesc), I32, D, U64, ctypes.c_uint32, V, V, I64, V, V]),
        "shgb_checkpoint_bytes": (I64, [I64, I32, I32, I32]),
        "shgb_step_checkpointed": (I32, [P(Model), P(StateDesc), I32, D, U64, I32, V, I64, V, V]),
        "shgb_population_adjoint_workspace": (I64, [I64, I32, I32]),
        "shgb_population_adjoint": (I32, [P(Model), P(StateDesc), V, I32, D, U64, I32, V, I64, V, V, I64, V]),
        "shgb_record_bytes": (I64, [I64, I32, I32, I32]),
        "shgb_step_recorded": (I32, [P(Model), P(StateDesc), I32, D, U64, I32, V, I64, V, I64, V, V]),
        "shgb_population_adjoint_recorded_workspace": (I64, [I64, I32, I32]),
        "shgb_population_adjoint_recorded": (I32, [P(Model), P(StateDesc), V, V, I32, D, U64, I32, V, I64, V, V, I64,
                                                   V]),
        "shgb_batch_table_bytes": (I64, [I32]),
        "shgb_batch_prepare": (I32, [P(Model), P(StateDesc), P(U64), I32, P(BatchConfig), V, I64, P(BatchDesc)]),
        "shgb_step_batched": (I32, [P(BatchDesc), I32, D, V, I64, V, V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = res, args
    sizes = (ctypes.c_int64 * 5)()
    lib.shgb_abi_sizes(ctypes.cast(sizes, ctypes.c_void_p))
    want = (ctypes.sizeof(Model), ctypes.sizeof(StateDesc), ctypes.sizeof(InitSpec), ctypes.sizeof(BatchConfig),
            ctypes.sizeof(BatchDesc))
    if tuple(sizes) != want:
        raise ImportError(f"libshgb ABI mismatch: C sizes {tuple(sizes)} vs binding {want}")
    return lib


_lib = _load()

EXPORTED = ("shgb_init_beams", "shgb_step_ensemble", "shgb_step_ensemble_scheme", "shgb_hop", "shgb_populations_workspace",
            "shgb_populations", "shgb_populations_noalloc", "shgb_population_stats",
            "shgb_reconstruct_workspace", "shgb_reconstruct", "shgb_reconstruct_workspace_mode",
            "shgb_reconstruct_mode", "shgb_philox",
            "shgb_strerror", "shgb_version", "shgb_abi_sizes", "shgb_batch_table_bytes", "shgb_batch_prepare",
            "shgb_step_batched", "shgb_population_tangent_workspace", "shgb_population_tangent",
            "shgb_checkpoint_bytes", "shgb_step_checkpointed", "shgb_population_adjoint_workspace",
            "shgb_population_adjoint", "shgb_record_bytes", "shgb_step_recorded",
            "shgb_population_adjoint_recorded_workspace", "shgb_population_adjoint_recorded")


def _check(fn, rc):
    if rc != SHGB_OK:
        raise ShgbError(fn, rc)


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def traj_fields(m):
    return 2 * m + m * (m + 1)


def nfields(m):
    return traj_fields(m) + SHGB_SCALAR_FIELDS


def make_model(d, mass, eps, A, B, C, D, lam=0.0, bath_omega=()):
    mdl = Model()
    mdl.kind, mdl.d = 1, int(d)
    mdl.mass, mdl.eps, mdl.A, mdl.B, mdl.C, mdl.D, mdl.lam = mass, eps, A, B, C, D, lam
    for k, w in enumerate(bath_omega):
        mdl.bath_omega[k] = float(w)
    return mdl


def make_linquad_model(eps, a, J, b0, b, H, gamma):
    """A linear-quadratic model (m = 2): arrays of shapes (n, 2), (n, 2, 2), (n,), (n, 2),
    (n, 2, 2) and gamma (n, n) complex with gamma[j, l] the rate from l to j."""
    import numpy as np
    a, J, b0, b, H = (np.asarray(v, dtype=np.float64) for v in (a, J, b0, b, H))
    G = np.asarray(gamma, dtype=np.complex128)
    n = a.shape[0]
    mdl = Model()
    mdl.kind, mdl.d, mdl.mass, mdl.eps = 2, 1, 1.0, float(eps)
    q = mdl.lq
    q.n_comp = n
    for l in range(n):
        q.b0[l] = b0[l]
        for i in range(2):
            q.a[l][i] = a[l, i]
            q.b[l][i] = b[l, i]
            for k in range(2):
                q.J[l][i][k] = J[l, i, k]
                q.H[l][i][k] = H[l, i, k]
        for j in range(n):
            q.gamma_re[j][l] = G[j, l].real
            q.gamma_im[j][l] = G[j, l].imag
    return mdl


def make_paper32_model(eps):
    """The nonlinear two-component system of eq:ex2 (see include/shgb.h)."""
    mdl = Model()
    mdl.kind, mdl.d, mdl.mass, mdl.eps = 3, 1, 1.0, float(eps)
    return mdl


def make_init_spec(q_mean, q_std, p_dist, p_a, p_b, comp0, a0=0.0):
    return InitSpec(q_mean, q_std, DIST[p_dist], p_a, p_b, comp0, a0)


class State:
    """Device beam state in the structure-of-arrays layout of include/shgb.h.

    ``precision`` "fp64": one float64 block of nfields(m) rows; "mixed": the
    trajectory rows (X, P, Zre, Zim) in a float32 block ``f32`` and the scalar
    rows (S, A, logw, phase, Lam, E) in a float64 block ``f64``.
    """

    def __init__(self, n, m, device="cuda", ld=None, beam_id_offset=0, precision="fp64"):
        self.n, self.m = int(n), int(m)
        self.ld = int(ld) if ld is not None else max(self.n, 1)
        self.beam_id_offset = int(beam_id_offset)
        self.precision = precision
        tf = traj_fields(m)
        if precision == "fp64":
            self.f64 = torch.zeros((nfields(m), self.ld), dtype=torch.float64, device=device)
            self.f32 = None
            self.traj, self.scal = self.f64[:tf], self.f64[tf:]
        elif precision == "mixed":
            self.f64 = torch.zeros((SHGB_SCALAR_FIELDS, self.ld), dtype=torch.float64, device=device)
            self.f32 = torch.zeros((tf, self.ld), dtype=torch.float32, device=device)
            self.traj, self.scal = self.f32, self.f64
        else:
            raise ValueError(f"precision must be 'fp64' or 'mixed', not {precision!r}")
        self.comp = torch.zeros(self.ld, dtype=torch.int32, device=device)
        self.nhop = torch.zeros(self.ld, dtype=torch.int32, device=device)  # uint32 in C

    def desc(self):
        return StateDesc(self.f64.data_ptr(), self.comp.data_ptr(), self.nhop.data_ptr(), self.n,
                         self.ld, self.beam_id_offset, self.m, PRECISION[self.precision],
                         0 if self.f32 is None else self.f32.data_ptr())

    @property
    def T(self):
        return self.m * (self.m + 1) // 2

    def traj_rows(self):
        """Row slices of the trajectory block (``traj``)."""
        m, T = self.m, self.T
        return dict(X=slice(0, m), P=slice(m, 2 * m), Zre=slice(2 * m, 2 * m + T),
                    Zim=slice(2 * m + T, 2 * m + 2 * T))

    SCALAR_ROWS = dict(S=0, Are=1, Aim=2, logw=3, phre=4, phim=5, Lam=6, E=7)


def new_diag(device="cuda"):
    return torch.zeros(SHGB_NDIAG, dtype=torch.int64, device=device)


def init_beams(model, spec, state, seed, stream=None):
    d = state.desc()
    _check("shgb_init_beams", _lib.shgb_init_beams(ctypes.byref(model), ctypes.byref(spec),
                                                   ctypes.byref(d), seed, _stream(stream)))


def step_ensemble(model, state, nsteps, dt, seed, diag=None, stream=None, scheme="rk4"):
    """Advance every beam by nsteps intervals of dt; scheme "rk4" (classical) or "rk3" (Kutta)."""
    d = state.desc()
    if scheme == "rk4":
        _check("shgb_step_ensemble", _lib.shgb_step_ensemble(ctypes.byref(model), ctypes.byref(d), int(nsteps),
                                                             float(dt), seed, _ptr(diag), _stream(stream)))
        return
    code = {"rk3": SHGB_SCHEME_RK3}[scheme]
    _check("shgb_step_ensemble_scheme", _lib.shgb_step_ensemble_scheme(ctypes.byref(model), ctypes.byref(d),
                                                                       int(nsteps), float(dt), seed, code,
                                                                       _ptr(diag), _stream(stream)))


def hop(model, state, idx, seed, diag=None, stream=None):
    d = state.desc()
    assert idx.dtype == torch.int32 and idx.is_contiguous()
    _check("shgb_hop", _lib.shgb_hop(ctypes.byref(model), ctypes.byref(d), _ptr(idx), idx.numel(), seed,
                                     _ptr(diag), _stream(stream)))


def populations_workspace(n, m):
    return int(_lib.shgb_populations_workspace(n, m))


def populations(model, state, out=None, work=None, diag=None, stream=None):
    """Raw per-component sums, a (4, 5) float64 device tensor (see include/shgb.h)."""
    dev = state.f64.device
    if out is None:
        out = torch.empty((SHGB_NCOMP, 5), dtype=torch.float64, device=dev)
    nb = populations_workspace(state.n, state.m)
    if work is None:
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=dev)
    d = state.desc()
    _check("shgb_populations", _lib.shgb_populations(ctypes.byref(model), ctypes.byref(d), _ptr(out),
                                                     _ptr(work), work.numel(), _ptr(diag), _stream(stream)))
    return out


def populations_noalloc(model, state, out, diag=None, stream=None):
    """``populations`` through the entry point that allocates nothing: partial sums in the
    library's own device array (see include/shgb.h).  out: a (4, 5) float64 device tensor."""
    assert out.dtype == torch.float64 and out.numel() >= SHGB_NCOMP * 5 and out.is_contiguous()
    d = state.desc()
    _check("shgb_populations_noalloc", _lib.shgb_populations_noalloc(ctypes.byref(model), ctypes.byref(d),
                                                                     _ptr(out), _ptr(diag), _stream(stream)))
    return out


FIELD_MODES = {"default": SHGB_FIELD_DEFAULT, "fp32": SHGB_FIELD_FP32_MATRIX}


def reconstruct_workspace(n, m, Q, mode="default"):
    return int(_lib.shgb_reconstruct_workspace_mode(n, m, Q, FIELD_MODES[mode]))


def reconstruct(model, state, points, out=None, work=None, stream=None, mode="default"):
    """Unnormalised sums per component at the points: a (4, Q) complex128 device tensor.
    mode "fp32" (m = 24): the exponents on the FP32 matrix cores (error stated in include/shgb.h)."""
    assert points.dtype == torch.float64 and points.is_contiguous() and points.shape[1] == state.m
    Q = points.shape[0]
    dev = state.f64.device
    if out is None:
        out = torch.empty((SHGB_NCOMP, Q, 2), dtype=torch.float64, device=dev)
    nb = reconstruct_workspace(state.n, state.m, Q, mode)
    if work is None:
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=dev)
    d = state.desc()
    _check("shgb_reconstruct_mode", _lib.shgb_reconstruct_mode(ctypes.byref(model), ctypes.byref(d), _ptr(points),
                                                               Q, _ptr(out), _ptr(work), work.numel(),
                                                               FIELD_MODES[mode], _stream(stream)))
    return torch.view_as_complex(out)


THETA_NAMES = ("A", "B", "C", "D", "p_mean")


def population_tangent_workspace(n):
    return int(_lib.shgb_population_tangent_workspace(int(n)))


def population_tangent(model, state, nsteps, dt, seed, dirs=range(5), out=None, work=None, diag=None,
                       stream=None):
    """Population sums and their derivatives along theta_j (see include/shgb.h): a (5, 4, 4)
    float64 device tensor [direction, component, (Re c, Im c, d Re c, d Im c)] summed over beams."""
    dev = state.f64.device
    if out is None:
        out = torch.zeros((5, SHGB_NCOMP, 4), dtype=torch.float64, device=dev)
    nb = population_tangent_workspace(state.n)
    if work is None:
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=dev)
    mask = 0
    for j in dirs:
        mask |= 1 << int(j)
    d = state.desc()
    _check("shgb_population_tangent", _lib.shgb_population_tangent(
        ctypes.byref(model), ctypes.byref(d), int(nsteps), float(dt), seed, mask, _ptr(out), _ptr(work),
        work.numel(), _ptr(diag), _stream(stream)))
    return out


DEFAULT_BATCH_CONFIG = (4, 2, 1)   # waves per block, blocks per CU, tiles per grab


def checkpoint_bytes(n, m, nsteps, every):
    return int(_lib.shgb_checkpoint_bytes(n, m, nsteps, every))


def step_checkpointed(model, state, nsteps, dt, seed, every=100, ckpt=None, diag=None, stream=None):
    """step_ensemble that also writes the state before every `every` intervals into a checkpoint
    buffer (a uint8 device tensor, allocated here if not given); returns the buffer."""
    nb = checkpoint_bytes(state.n, state.m, nsteps, every)
    if ckpt is None:
        ckpt = torch.empty(max(nb, 8), dtype=torch.uint8, device=state.f64.device)
    d = state.desc()
    _check("shgb_step_checkpointed", _lib.shgb_step_checkpointed(ctypes.byref(model), ctypes.byref(d), nsteps,
                                                                 float(dt), seed, every, _ptr(ckpt), ckpt.numel(),
                                                                 _ptr(diag), _stream(stream)))
    return ckpt


def population_adjoint_workspace(n, m, every):
    return int(_lib.shgb_population_adjoint_workspace(n, m, every))


def population_adjoint(model, state, ckpt, nsteps, dt, seed, cot, n_traj, every=100, out=None, work=None,
                       stream=None):
    """Reverse sweep: (dL/dA, dL/dB, dL/dC, dL/dD, dL/dp_mean, L) as a device tensor of 6, for
    L = sum_i cot[2i] Re U_i + cot[2i+1] Im U_i (cot: 8 doubles on the device)."""
    dev = state.f64.device
    assert cot.dtype == torch.float64 and cot.is_contiguous() and cot.numel() >= 2 * SHGB_NCOMP
    if out is None:
        out = torch.empty(6, dtype=torch.float64, device=dev)
    nb = population_adjoint_workspace(state.n, state.m, every)
    if work is None:
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=dev)
    d = state.desc()
    _check("shgb_population_adjoint", _lib.shgb_population_adjoint(
        ctypes.byref(model), ctypes.byref(d), _ptr(ckpt), nsteps, float(dt), seed, every, _ptr(cot), int(n_traj),
        _ptr(out), _ptr(work), work.numel(), _stream(stream)))
    return out


def record_bytes(n, m, nsteps, every):
    return int(_lib.shgb_record_bytes(n, m, nsteps, every))


def step_recorded(model, state, nsteps, dt, seed, every=100, ckpt=None, recs=None, diag=None, stream=None):
    """step_checkpointed that also keeps every interval's stage records (d > 1) in recs (a float64
    device tensor of record_bytes / 8 elements, allocated here if not given); returns (ckpt, recs)."""
    dev = state.f64.device
    nb = checkpoint_bytes(state.n, state.m, nsteps, every)
    if ckpt is None:
        ckpt = torch.empty(max(nb, 8), dtype=torch.uint8, device=dev)
    rb = record_bytes(state.n, state.m, nsteps, every)
    if recs is None:
        recs = torch.empty(max(rb, 8) // 8, dtype=torch.float64, device=dev)
    assert recs.dtype == torch.float64 and recs.is_contiguous()
    d = state.desc()
    _check("shgb_step_recorded", _lib.shgb_step_recorded(ctypes.byref(model), ctypes.byref(d), nsteps, float(dt),
                                                         seed, every, _ptr(ckpt), ckpt.numel(), _ptr(recs),
                                                         recs.numel() * 8, _ptr(diag), _stream(stream)))
    return ckpt, recs


def population_adjoint_recorded_workspace(n, m, every):
    return int(_lib.shgb_population_adjoint_recorded_workspace(n, m, every))


def population_adjoint_recorded(model, state, ckpt, recs, nsteps, dt, seed, cot, n_traj, every=100, out=None,
                                work=None, stream=None):
    """population_adjoint from the records step_recorded kept (no replay of the segments)."""
    dev = state.f64.device
    assert cot.dtype == torch.float64 and cot.is_contiguous() and cot.numel() >= 2 * SHGB_NCOMP
    if out is None:
        out = torch.empty(6, dtype=torch.float64, device=dev)
    nb = population_adjoint_recorded_workspace(state.n, state.m, every)
    if work is None:
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=dev)
    d = state.desc()
    _check("shgb_population_adjoint_recorded", _lib.shgb_population_adjoint_recorded(
        ctypes.byref(model), ctypes.byref(d), _ptr(ckpt), _ptr(recs), nsteps, float(dt), seed, every, _ptr(cot),
        int(n_traj), _ptr(out), _ptr(work), work.numel(), _stream(stream)))
    return out


class Batch:
    """Instances (model, state, seed) advanced together by one persistent launch.

    The instance table is written on the host by shgb_batch_prepare and kept
    in device memory by this object, with the queue's work buffer; ``step``
    is one call of shgb_step_batched (capturable in a HIP graph).
    """

    def __init__(self, models, states, seeds, config=DEFAULT_BATCH_CONFIG, device="cuda"):
        n = len(models)
        assert n == len(states) == len(seeds) and n >= 1
        self.models, self.states, self.seeds = list(models), list(states), [int(x) for x in seeds]
        self.config = config if isinstance(config, BatchConfig) else BatchConfig(*config)
        nbytes = int(_lib.shgb_batch_table_bytes(n))
        host = (ctypes.c_uint8 * nbytes)()
        self._models = (Model * n)(*self.models)
        self._states = (StateDesc * n)(*[st.desc() for st in self.states])
        self._seeds = (ctypes.c_uint64 * n)(*self.seeds)
        self.desc = BatchDesc()
        _check("shgb_batch_prepare", _lib.shgb_batch_prepare(self._models, self._states, self._seeds, n,
                                                             ctypes.byref(self.config), host, nbytes,
                                                             ctypes.byref(self.desc)))
        self.table = torch.frombuffer(bytearray(bytes(host)), dtype=torch.uint8).to(device)
        self.desc.table = self.table.data_ptr()
        self.work = torch.zeros(SHGB_BATCH_WORK_BYTES, dtype=torch.uint8, device=device)

    @property
    def total_tiles(self):
        return int(self.desc.total_tiles)

    def step(self, nsteps, dt, diag=None, stream=None):
        _check("shgb_step_batched", _lib.shgb_step_batched(ctypes.byref(self.desc), int(nsteps), float(dt),
                                                           _ptr(self.work), self.work.numel(), _ptr(diag),
                                                           _stream(stream)))


def philox(seed, counters, stream=None):
    """Raw Philox4x64-10 blocks for (n, 4) counters (int64 tensor holding uint64 bits)."""
    out = torch.empty_like(counters)
    _check("shgb_philox", _lib.shgb_philox(seed, _ptr(counters), _ptr(out), counters.shape[0], _stream(stream)))
    return out


def population_stats(sums, n_traj, out=None, stream=None):
    """Means and standard errors per component from the raw sums of ``populations`` (a device
    tensor of 4 x 5 doubles), computed on the device: a (4, 4) float64 tensor of
    (Re mean, Im mean, SE of Re, SE of Im)."""
    assert sums.dtype == torch.float64 and sums.is_contiguous() and sums.is_cuda
    if out is None:
        out = torch.empty((SHGB_NCOMP, 4), dtype=torch.float64, device=sums.device)
    _check("shgb_population_stats", _lib.shgb_population_stats(_ptr(sums), int(n_traj), _ptr(out),
                                                                 _stream(stream)))
    return out


def population_mean_se(sums, n_traj):
    """(mean, SE) as complex host numpy arrays of 4, from ``population_stats`` (the sums may be a
    device tensor or host values, which are copied to the device)."""
    if not torch.is_tensor(sums):
        sums = torch.as_tensor(sums, dtype=torch.float64)
    if not sums.is_cuda:
        sums = sums.to(dtype=torch.float64, device="cuda").contiguous()
    st = population_stats(sums, n_traj).cpu().numpy()
    return st[:, 0] + 1j * st[:, 1], st[:, 2] + 1j * st[:, 3]


def unpack(state):
    """Host copy of the state as full matrices in float64: dict of numpy arrays."""
    import numpy as np
    n, m = state.n, state.m
    t = state.traj[:, :n].double().cpu().numpy()
    f = state.scal[:, :n].cpu().numpy()
    r, c = state.traj_rows(), State.SCALAR_ROWS
    iu = np.triu_indices(m)
    Z = np.zeros((n, m, m), dtype=np.complex128)
    Z[:, iu[0], iu[1]] = (t[r["Zre"]] + 1j * t[r["Zim"]]).T
    Z[:, iu[1], iu[0]] = (t[r["Zre"]] + 1j * t[r["Zim"]]).T
    return dict(X=t[r["X"]].T.copy(), P=t[r["P"]].T.copy(), Z=Z, S=f[c["S"]].copy(),
                A=f[c["Are"]] + 1j * f[c["Aim"]], logw=f[c["logw"]].copy(),
                phase=f[c["phre"]] + 1j * f[c["phim"]], Lam=f[c["Lam"]].copy(), E=f[c["E"]].copy(),
                comp=state.comp[:n].cpu().numpy().astype(np.int64),
                nhop=state.nhop[:n].cpu().numpy().astype(np.int64) & 0xFFFFFFFF)


def pack(arrays, device="cuda", beam_id_offset=0, ld=None, precision="fp64"):
    """Device state from host arrays with the keys ``unpack`` returns (trajectory
    values rounded to float32 for a mixed state)."""
    import numpy as np
    X = np.asarray(arrays["X"], dtype=np.float64)
    n, m = X.shape
    st = State(n, m, device=device, ld=ld, beam_id_offset=beam_id_offset, precision=precision)
    r, c = st.traj_rows(), State.SCALAR_ROWS
    iu = np.triu_indices(m)
    t = np.zeros((traj_fields(m), st.ld))
    t[r["X"], :n] = X.T
    t[r["P"], :n] = np.asarray(arrays["P"]).T
    Z = np.asarray(arrays["Z"])
    t[r["Zre"], :n] = Z[:, iu[0], iu[1]].real.T
    t[r["Zim"], :n] = Z[:, iu[0], iu[1]].imag.T
    f = np.zeros((SHGB_SCALAR_FIELDS, st.ld))
    f[c["S"], :n] = arrays["S"]
    f[c["Are"], :n] = np.real(arrays["A"])
    f[c["Aim"], :n] = np.imag(arrays["A"])
    f[c["logw"], :n] = arrays["logw"]
    f[c["phre"], :n] = np.real(arrays["phase"])
    f[c["phim"], :n] = np.imag(arrays["phase"])
    f[c["Lam"], :n] = arrays["Lam"]
    f[c["E"], :n] = arrays["E"]
    st.traj.copy_(torch.from_numpy(t).to(st.traj.dtype))
    st.scal.copy_(torch.from_numpy(f))
    st.comp[:n].copy_(torch.from_numpy(np.asarray(arrays["comp"], dtype=np.int32)))
    st.nhop[:n].copy_(torch.from_numpy(np.asarray(arrays["nhop"], dtype=np.int64).astype(np.uint32).view(np.int32)))
    return st
