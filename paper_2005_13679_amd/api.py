"""Python API over libmc: torch supplies device memory and the current stream;
every step of the computation runs in the library's HIP kernels."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require(t: torch.Tensor, name: str, dtype, device, numel=None, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


# ---------------------------------------------------------------------------
# host combinatorics
# ---------------------------------------------------------------------------

def dim(N: int, M: int) -> int:
    """N_c(N, M) = C(N+M-1, N) (Eq. nc)."""
    d = L.load().mc_dim(N, M)
    if d < 0:
        L.check(int(d), "mc_dim")
    return int(d)


def hash_occ(N: int, M: int, occ) -> int:
    """Index of one configuration (host)."""
    a = np.ascontiguousarray(occ, dtype=np.int32)
    if a.size != M:
        raise ValueError("occupation vector must have M entries")
    out = ctypes.c_int64()
    L.check(L.load().mc_hash(N, M, a.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)), "mc_hash")
    return int(out.value)


def unhash(N: int, M: int, index: int) -> np.ndarray:
    """Configuration of one index (host)."""
    out = np.empty(M, dtype=np.int32)
    L.check(L.load().mc_unhash(N, M, int(index), out.ctypes.data_as(ctypes.c_void_p)), "mc_unhash")
    return out


def tables_size(N: int, M: int) -> L.TableSizes:
    s = L.TableSizes()
    L.check(L.load().mc_tables_size(N, M, ctypes.byref(s)), "mc_tables_size")
    return s


def tables_bytes(N: int, M: int, form: str = "paper", double_jumps: bool = True) -> int:
    """Device bytes of the tables of (N, M) (the double-jump map at its
    largest tiled size)."""
    out = ctypes.c_int64()
    L.check(L.load().mc_tables_bytes(N, M, L.FORMS[form], int(bool(double_jumps)),
                                     ctypes.byref(out)), "mc_tables_bytes")
    return int(out.value)


def choose_double_jumps(shapes, budget_bytes: float, form: str = "paper") -> list[bool]:
    """Which instances [(N, M), ...] keep a double-jump map within
    `budget_bytes` of map memory (smallest maps first); the rest chain
    single jumps."""
    n = len(shapes)
    Ns = np.ascontiguousarray([s[0] for s in shapes], dtype=np.int32)
    Ms = np.ascontiguousarray([s[1] for s in shapes], dtype=np.int32)
    keep = np.zeros(n, dtype=np.int32)
    L.check(L.load().mc_choose_double_jumps(n, Ns.ctypes.data_as(ctypes.c_void_p),
                                            Ms.ctypes.data_as(ctypes.c_void_p), L.FORMS[form],
                                            float(budget_bytes),
                                            keep.ctypes.data_as(ctypes.c_void_p)),
            "mc_choose_double_jumps")
    return [bool(k) for k in keep]


def apply_stream_columns(M: int, form: str = "reduced") -> tuple[int, int]:
    """(jump slots per row, slots a tile whose rows reach every removal pair
    reads from the tables) of the apply through the double-jump map of
    `form` ("paper" or "reduced")."""
    slots, cols = L.c_i32(), L.c_i32()
    L.check(L.load().mc_apply_stream_columns(M, L.FORMS[form], ctypes.byref(slots),
                                             ctypes.byref(cols)), "mc_apply_stream_columns")
    return int(slots.value), int(cols.value)


def workspace_size(N: int, M: int, op: int) -> int:
    b = L.c_sz()
    L.check(L.load().mc_workspace_size(N, M, op, ctypes.byref(b)), "mc_workspace_size")
    return int(b.value)


# ---------------------------------------------------------------------------
# tables
# ---------------------------------------------------------------------------

class Tables:
    """Hashing table and jump maps of the space (N, M) on one device.

    Buffers are torch tensors owned by this object; ``c`` is the C descriptor
    passed to the library."""

    def __init__(self, N: int, M: int, device=None, double_jumps: bool = True,
                 form: str = "paper"):
        device = torch.device(device if device is not None else "cuda")
        if device.type != "cuda":
            raise ValueError("tables live in GPU memory")
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        if form not in L.FORMS:
            raise ValueError(f"form must be one of {sorted(L.FORMS)}")
        self.N, self.M, self.device = int(N), int(M), device
        self.form = form
        sz = tables_size(N, M)
        self.sizes = sz
        self.dim, self.tiles = int(sz.dim), int(sz.tiles)

        def buf(nbytes, dtype=torch.uint8):
            n = max(1, int(nbytes) // torch.empty((), dtype=dtype).element_size())
            return torch.empty(n, dtype=dtype, device=device)

        self.binom = buf(sz.binom_bytes, torch.int64)
        self.occ = buf(sz.occ_bytes_total, torch.uint8 if sz.occ_bytes == 1 else torch.int16)
        self.t1 = buf(sz.t1_bytes, torch.int32)
        self.pmask = buf(sz.pmask_bytes, torch.int64)
        self.t2_off = buf(sz.t2_off_bytes, torch.int64)
        self.t2 = None
        c = L.CTables()
        c.N, c.M, c.dim, c.tiles = self.N, self.M, self.dim, self.tiles
        c.binom_d = self.binom.data_ptr()
        c.occ_d = self.occ.data_ptr()
        c.t1_d = self.t1.data_ptr()
        c.pmask_d = self.pmask.data_ptr()
        c.t2_off_d = self.t2_off.data_ptr()
        c.t2_d = None
        c.t2_entries = 0
        c.t2_required = -1
        c.form = L.FORMS[form]
        self.c = c
        with torch.cuda.device(device):
            L.check(L.load().mc_build_jump_tables(N, M, ctypes.byref(c), _stream(device)),
                    "mc_build_jump_tables")
            if double_jumps:
                self.build_double_jumps()
        self._ws = {}

    @property
    def t2_required(self) -> int:
        return int(self.c.t2_required)

    def build_double_jumps(self):
        need = self.t2_required
        self.t2 = torch.empty(max(1, need), dtype=torch.int32, device=self.device)
        self.c.t2_d = self.t2.data_ptr()
        self.c.t2_entries = need
        with torch.cuda.device(self.device):
            L.check(L.load().mc_build_double_jumps(self.N, self.M, ctypes.byref(self.c),
                                                   _stream(self.device)),
                    "mc_build_double_jumps")

    def workspace(self, op: int) -> torch.Tensor:
        ws = self._ws.get(op)
        if ws is None:
            nbytes = workspace_size(self.N, self.M, op)
            ws = torch.empty(max(16, nbytes), dtype=torch.uint8, device=self.device)
            self._ws[op] = ws
        return ws

    def nbytes(self) -> dict:
        d = {
            "binom": self.binom.numel() * 8,
            "occ": self.occ.numel() * self.occ.element_size(),
            "t1": self.t1.numel() * 4,
            "pmask": self.pmask.numel() * 8,
            "t2_off": self.t2_off.numel() * 8,
            "t2": 0 if self.t2 is None else self.t2.numel() * 4,
        }
        return d

    # --- readback helpers (testing / inspection) --------------------------
    def occupations(self) -> np.ndarray:
        """Row-major (D, M) occupation table, copied to the host."""
        o = self.occ.cpu().numpy()
        if o.dtype == np.int16:
            o = o.view(np.uint16)
        o = o.astype(np.int64).reshape(self.tiles, self.M, L.MC_TILE)
        return o.transpose(0, 2, 1).reshape(-1, self.M)[: self.dim]

    def single_jumps(self) -> np.ndarray:
        """Dense (D, M, M) single-jump map, copied to the host."""
        t = self.t1.cpu().numpy().reshape(self.tiles, self.M, self.M, L.MC_TILE)
        return t.transpose(0, 3, 1, 2).reshape(-1, self.M, self.M)[: self.dim]


def build_tables(N: int, M: int, device=None, double_jumps: bool = True,
                 form: str = "paper") -> Tables:
    """Tables of (N, M).  form="paper": the paper's double-jump map (M*M
    slots per removal pair); form="reduced": only the true double jumps, and
    H.C runs in the case-split form.  double_jumps=False builds no map (the
    apply then chains single jumps)."""
    return Tables(N, M, device, double_jumps, form)


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------

class DirectSpace:
    """The space (N, M) with no table: ``apply_H`` on it evaluates H.C
    table-free (mc_apply_H_direct), and as a batch item it runs table-free in
    the persistent kernel.  ``c`` is a table descriptor holding sizes only."""

    form = "direct"
    t2 = None

    def __init__(self, N: int, M: int, device=None):
        device = torch.device(device if device is not None else "cuda")
        if device.type != "cuda":
            raise ValueError("the table-free apply runs on the GPU")
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.N, self.M, self.device = int(N), int(M), device
        self.dim = dim(N, M)
        self.tiles = (self.dim + 63) // 64
        c = L.CTables()
        c.N, c.M, c.dim, c.tiles = self.N, self.M, self.dim, self.tiles
        c.t2_required = -1
        self.c = c
        self._ws = None

    def workspace(self, op: int) -> torch.Tensor:
        # the table-free density matrices have workspaces of their own
        op = {L.MC_OP_RHO1: L.MC_OP_RHO1_DIRECT, L.MC_OP_RHO2: L.MC_OP_RHO2_DIRECT}.get(op, op)
        if op not in (L.MC_OP_APPLY, L.MC_OP_RHO1_DIRECT, L.MC_OP_RHO2_DIRECT):
            raise ValueError("a table-free space supports H.C, rho1 and rho2")
        if self._ws is None:
            self._ws = {}
        ws = self._ws.get(op)
        if ws is None:
            ws = torch.empty(max(16, workspace_size(self.N, self.M, op)), dtype=torch.uint8,
                             device=self.device)
            self._ws[op] = ws
        return ws

    def nbytes(self) -> dict:
        return {}


def _as_dev(x, device, shape=None) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.asarray(x))
    x = x.to(device=device, dtype=torch.complex128)
    if shape is not None:
        x = x.reshape(shape)
    return x.contiguous()


def apply_H(h, g, C: torch.Tensor, tables, out: torch.Tensor | None = None) -> torch.Tensor:
    """HC = H . C (Eq. Haction) on the GPU through the jump maps (Tables), or
    table-free (DirectSpace)."""
    if isinstance(tables, DirectSpace):
        return apply_H_direct(h, g, C, tables.N, tables.M, out=out, _space=tables)
    N, M, dev = tables.N, tables.M, tables.device
    h = _as_dev(h, dev, (M, M))
    g = _as_dev(g, dev, (M, M, M, M))
    _require(C, "C", torch.complex128, dev, numel=tables.dim)
    if out is None:
        out = torch.empty_like(C)
    _require(out, "out", torch.complex128, dev, numel=tables.dim)
    ws = tables.workspace(L.MC_OP_APPLY)
    with torch.cuda.device(dev):
        L.check(L.load().mc_apply_H(N, M, _ptr(h), _ptr(g), ctypes.byref(tables.c), _ptr(C),
                                    _ptr(out), _ptr(ws), ws.numel(), _stream(dev)), "mc_apply_H")
    return out


def apply_H_sparse(h, g, C: torch.Tensor, tables: Tables,
                   out: torch.Tensor | None = None) -> torch.Tensor:
    """HC = H . C in the case-split form, gathering only the jumps whose
    constants are nonzero (reduced-form tables; pays when most of g
    vanishes, e.g. a momentum-conserving interaction)."""
    N, M, dev = tables.N, tables.M, tables.device
    h = _as_dev(h, dev, (M, M))
    g = _as_dev(g, dev, (M, M, M, M))
    _require(C, "C", torch.complex128, dev, numel=tables.dim)
    if out is None:
        out = torch.empty_like(C)
    _require(out, "out", torch.complex128, dev, numel=tables.dim)
    ws = tables.workspace(L.MC_OP_APPLY)
    with torch.cuda.device(dev):
        L.check(L.load().mc_apply_H_sparse(N, M, _ptr(h), _ptr(g), ctypes.byref(tables.c),
                                           _ptr(C), _ptr(out), _ptr(ws), ws.numel(),
                                           _stream(dev)), "mc_apply_H_sparse")
    return out


_direct_spaces: dict = {}


def apply_H_direct(h, g, C: torch.Tensor, N: int, M: int,
                   out: torch.Tensor | None = None, _space: DirectSpace | None = None) -> torch.Tensor:
    """HC = H . C with no table: occupations and jump targets of every row
    from its index in closed form (M <= 8, dim < 2^31).  Device memory is C,
    out and a small workspace only."""
    if not isinstance(C, torch.Tensor):
        raise TypeError("C must be a torch.Tensor")
    dev = C.device
    sp = _space
    if sp is None:
        sp = _direct_spaces.get((dev, N, M))
        if sp is None:
            sp = _direct_spaces[(dev, N, M)] = DirectSpace(N, M, dev)
    D = sp.dim
    h = _as_dev(h, dev, (M, M))
    g = _as_dev(g, dev, (M, M, M, M))
    _require(C, "C", torch.complex128, dev, numel=D)
    if out is None:
        out = torch.empty_like(C)
    _require(out, "out", torch.complex128, dev, numel=D)
    ws = sp.workspace(L.MC_OP_APPLY)
    with torch.cuda.device(dev):
        L.check(L.load().mc_apply_H_direct(N, M, _ptr(h), _ptr(g), _ptr(C), _ptr(out), _ptr(ws),
                                           ws.numel(), _stream(dev)), "mc_apply_H_direct")
    return out


def apply_H_adjoint(h, g, C: torch.Tensor, tables, out: torch.Tensor | None = None) -> torch.Tensor:
    """H^dagger . C (h -> h^dagger, g_ksql -> conj(g_lqsk)), through the jump
    maps (Tables) or table-free (DirectSpace)."""
    N, M, dev = tables.N, tables.M, tables.device
    h = _as_dev(h, dev, (M, M))
    g = _as_dev(g, dev, (M, M, M, M))
    _require(C, "C", torch.complex128, dev, numel=tables.dim)
    if out is None:
        out = torch.empty_like(C)
    _require(out, "out", torch.complex128, dev, numel=tables.dim)
    ws = tables.workspace(L.MC_OP_APPLY)
    with torch.cuda.device(dev):
        if isinstance(tables, DirectSpace):
            L.check(L.load().mc_apply_H_direct_adjoint(N, M, _ptr(h), _ptr(g), _ptr(C), _ptr(out),
                                                       _ptr(ws), ws.numel(), _stream(dev)),
                    "mc_apply_H_direct_adjoint")
        else:
            L.check(L.load().mc_apply_H_adjoint(N, M, _ptr(h), _ptr(g), ctypes.byref(tables.c),
                                                _ptr(C), _ptr(out), _ptr(ws), ws.numel(),
                                                _stream(dev)), "mc_apply_H_adjoint")
    return out


def is_hermitian(h, g, M: int, device) -> bool:
    """True if h = h^dagger and g_ksql = conj(g_lqsk) elementwise (then
    H^dagger = H); one small kernel and a 4-byte read back."""
    h = _as_dev(h, device, (M, M))
    g = _as_dev(g, device, (M, M, M, M))
    flag = torch.empty(1, dtype=torch.int32, device=device)
    with torch.cuda.device(device):
        L.check(L.load().mc_is_hermitian(M, _ptr(h), _ptr(g), _ptr(flag), _stream(device)),
                "mc_is_hermitian")
    return bool(flag.item())


def zaxpby(x: torch.Tensor, a: torch.Tensor | None = None, y: torch.Tensor | None = None,
           b: torch.Tensor | None = None, scale: float = 1.0, conj_a=False, conj_x=False,
           conj_b=False, conj_y=False, out: torch.Tensor | None = None) -> torch.Tensor:
    """out = scale * (op(a) op(x) + op(b) op(y)) with 0-d device scalars a, b."""
    dev = x.device
    _require(x, "x", torch.complex128, dev)
    if y is not None:
        _require(y, "y", torch.complex128, dev, numel=x.numel())
    for name, v in (("a", a), ("b", b)):
        if v is not None:
            _require(v, name, torch.complex128, dev, numel=1)
    if out is None:
        out = torch.empty_like(x)
    _require(out, "out", torch.complex128, dev, numel=x.numel())
    flags = ((L.MC_CONJ_A if conj_a else 0) | (L.MC_CONJ_X if conj_x else 0)
             | (L.MC_CONJ_B if conj_b else 0) | (L.MC_CONJ_Y if conj_y else 0))
    nul = ctypes.c_void_p(None)
    with torch.cuda.device(dev):
        L.check(L.load().mc_zaxpby(x.numel(), _ptr(a) if a is not None else nul, _ptr(x),
                                   _ptr(b) if b is not None else nul,
                                   _ptr(y) if y is not None else nul, float(scale), flags,
                                   _ptr(out), _stream(dev)), "mc_zaxpby")
    return out


def rho1(C: torch.Tensor, tables: Tables, out: torch.Tensor | None = None) -> torch.Tensor:
    """One-body reduced density matrix rho_kl = <a+_k a_l> (Eq. rho1), through
    the single-jump map (Tables) or table-free (DirectSpace)."""
    M, dev = tables.M, tables.device
    _require(C, "C", torch.complex128, dev, numel=tables.dim)
    if out is None:
        out = torch.empty((M, M), dtype=torch.complex128, device=dev)
    _require(out, "out", torch.complex128, dev, numel=M * M)
    ws = tables.workspace(L.MC_OP_RHO1)
    if isinstance(tables, DirectSpace):
        with torch.cuda.device(dev):
            L.check(L.load().mc_rho1_direct(tables.N, M, _ptr(C), _ptr(out), _ptr(ws), ws.numel(),
                                            _stream(dev)), "mc_rho1_direct")
        return out
    with torch.cuda.device(dev):
        L.check(L.load().mc_rho1(tables.N, M, ctypes.byref(tables.c), _ptr(C), _ptr(out),
                                 _ptr(ws), ws.numel(), _stream(dev)), "mc_rho1")
    return out


def rho2(C: torch.Tensor, tables: Tables, out: torch.Tensor | None = None) -> torch.Tensor:
    """Two-body reduced density matrix rho_ksql = <a+_k a+_s a_q a_l> (Eq. rho2),
    through the double-jump map (Tables) or table-free (DirectSpace)."""
    M, dev = tables.M, tables.device
    _require(C, "C", torch.complex128, dev, numel=tables.dim)
    if out is None:
        out = torch.empty((M, M, M, M), dtype=torch.complex128, device=dev)
    _require(out, "out", torch.complex128, dev, numel=M ** 4)
    ws = tables.workspace(L.MC_OP_RHO2)
    if isinstance(tables, DirectSpace):
        with torch.cuda.device(dev):
            L.check(L.load().mc_rho2_direct(tables.N, M, _ptr(C), _ptr(out), _ptr(ws), ws.numel(),
                                            _stream(dev)), "mc_rho2_direct")
        return out
    with torch.cuda.device(dev):
        L.check(L.load().mc_rho2(tables.N, M, ctypes.byref(tables.c), _ptr(C), _ptr(out),
                                 _ptr(ws), ws.numel(), _stream(dev)), "mc_rho2")
    return out


_dot_ws = {}


def zdotc(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """sum(conj(x) * y) with a fixed-order reduction; returns a 0-d device tensor."""
    dev = x.device
    _require(x, "x", torch.complex128, dev)
    _require(y, "y", torch.complex128, dev, numel=x.numel())
    if out is None:
        out = torch.empty((), dtype=torch.complex128, device=dev)
    ws = _dot_ws.get(dev)
    if ws is None:
        ws = torch.empty((L.MC_DOT_BLOCKS + 1) * 16, dtype=torch.uint8, device=dev)
        _dot_ws[dev] = ws
    with torch.cuda.device(dev):
        L.check(L.load().mc_zdotc(x.numel(), _ptr(x), _ptr(y), _ptr(out), _ptr(ws), ws.numel(),
                                  _stream(dev)), "mc_zdotc")
    return out


def hash_batch(occ: torch.Tensor, tables: Tables) -> torch.Tensor:
    """Indices of many configurations (int32 occupations, shape (count, M))."""
    dev = tables.device
    _require(occ, "occ", torch.int32, dev)
    count = occ.numel() // tables.M
    out = torch.empty(count, dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        L.check(L.load().mc_hash_batch(tables.N, tables.M, ctypes.byref(tables.c), _ptr(occ),
                                       _ptr(out), count, _stream(dev)), "mc_hash_batch")
    return out


def unhash_batch(idx: torch.Tensor, tables: Tables) -> torch.Tensor:
    """Configurations of many indices (int64), shape (count, M) int32."""
    dev = tables.device
    _require(idx, "idx", torch.int64, dev)
    out = torch.empty((idx.numel(), tables.M), dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        L.check(L.load().mc_unhash_batch(tables.N, tables.M, ctypes.byref(tables.c), _ptr(idx),
                                         _ptr(out), idx.numel(), _stream(dev)), "mc_unhash_batch")
    return out


def t2_lookup(queries: torch.Tensor, tables: Tables) -> torch.Tensor:
    """Double-jump entries for (row, k, s, q, l) queries, shape (count, 5) int64."""
    dev = tables.device
    _require(queries, "queries", torch.int64, dev)
    count = queries.numel() // 5
    out = torch.empty(count, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        L.check(L.load().mc_t2_lookup(tables.N, tables.M, ctypes.byref(tables.c), _ptr(queries),
                                      _ptr(out), count, _stream(dev)), "mc_t2_lookup")
    return out
