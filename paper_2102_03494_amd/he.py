"""Thin Python binding of the C ABI (include/ffconv_he.h).

Argument marshalling only: device buffers are torch tensors (dtype int64
holding the uint64 residues bit for bit) whose data pointers are handed to
the library together with torch's current HIP stream.  Every computation runs
in the library's HIP kernels.  Scale bookkeeping (a float per ciphertext) is
kept here, on the host, with the same IEEE operations as the layer contract
documents.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import HeConvDesc, HeCounts, HeParams


class HEError(RuntimeError):
    pass


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise HEError("expected a device tensor")
    if not t.is_contiguous():
        raise HEError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    """uint64 numpy array -> int64 device tensor with the same bits."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a.copy()).to(device)


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def galois_for_rotation(k: int, n: int) -> int:
    slots = n // 2
    return pow(5, k % slots, 2 * n)


@dataclass
class Ct:
    """A batch of ciphertexts [count][2][level][N] on the device plus its scale."""
    data: torch.Tensor
    scale: float

    @property
    def level(self) -> int:
        return self.data.shape[-2]

    @property
    def count(self) -> int:
        return int(np.prod(self.data.shape[:-3], dtype=np.int64)) if self.data.dim() > 3 else 1


class Graph:
    """An instantiated HIP graph of library calls (HEContext.capture)."""

    def __init__(self, ctx, handle: ctypes.c_void_p):
        self.ctx = ctx
        self.h = handle

    def launch(self):
        self.ctx._check(self.ctx.lib.he_graph_launch(self.h, _stream()), "he_graph_launch")

    def close(self):
        if self.h:
            self.ctx.lib.he_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HEContext:
    def __init__(self, n: int, q_bits, p_bits: int, workspace_bytes: int = 0, tuned: bool = True):
        """A library context for ring dimension n, ciphertext primes of the
        given bit sizes and a special prime of p_bits.  With `tuned`, the
        autotuner's cached schedule for this ring (tune.py) is applied;
        tuning_source tells whether it came from the cache or the cost model."""
        self.lib = _lib.lib()
        self.n = int(n)
        self.q_bits = tuple(int(b) for b in q_bits)
        self.p_bits = int(p_bits)
        self.L = len(self.q_bits)
        prm = HeParams()
        prm.n = self.n
        prm.n_q = self.L
        for i, b in enumerate(self.q_bits):
            prm.q_bits[i] = b
        prm.p_bits = self.p_bits
        self._params = prm
        h = ctypes.c_void_p()
        self._check(self.lib.he_ctx_create(ctypes.byref(prm), ctypes.byref(h)), "he_ctx_create", ctx=None)
        self.h = h
        out = (ctypes.c_uint64 * (self.L + 1))()
        self._check(self.lib.he_ctx_moduli(self.h, out), "he_ctx_moduli")
        self.moduli = [int(v) for v in out]
        self.q = self.moduli[: self.L]
        self.p = self.moduli[self.L]
        self.tuning_source = "cost model"
        if tuned:
            from .tune import apply
            self.tuning_source = apply(self)
        if workspace_bytes:
            self.reserve(workspace_bytes)

    # ---- plumbing --------------------------------------------------------
    def _check(self, rc: int, what: str, ctx="self"):
        if rc != 0:
            msg = ""
            if ctx == "self" and getattr(self, "h", None) is not None:
                msg = self.lib.he_last_error(self.h).decode()
            raise HEError(f"{what} failed with code {rc}: {msg}")

    def close(self):
        if getattr(self, "h", None) is not None:
            self.lib.he_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def params_moduli(n, q_bits, p_bits) -> list[int]:
        lib = _lib.lib()
        prm = HeParams()
        prm.n = n
        prm.n_q = len(q_bits)
        for i, b in enumerate(q_bits):
            prm.q_bits[i] = b
        prm.p_bits = p_bits
        out = (ctypes.c_uint64 * (len(q_bits) + 1))()
        rc = lib.he_params_moduli(ctypes.byref(prm), out)
        if rc != 0:
            raise HEError(f"he_params_moduli failed with code {rc}")
        return [int(v) for v in out]

    def reserve(self, nbytes: int):
        self._check(self.lib.he_ctx_reserve(self.h, ctypes.c_size_t(int(nbytes))), "he_ctx_reserve")

    def workspace_need(self, count: int, level: int) -> int:
        return int(self.lib.he_ctx_workspace_need(self.h, count, level))

    def set_tuning(self, knob: str, level: int, value: int):
        self._check(self.lib.he_ctx_set_tuning(self.h, knob.encode(), level, value), "he_ctx_set_tuning")

    def get_tuning(self, knob: str, level: int) -> int:
        v = int(self.lib.he_ctx_get_tuning(self.h, knob.encode(), level))
        if v < 0:
            self._check(v, "he_ctx_get_tuning")
        return v

    def empty_ct(self, count: int, level: int) -> torch.Tensor:
        return torch.empty((count, 2, level, self.n), dtype=torch.int64, device="cuda")

    def last_counts(self) -> dict:
        c = HeCounts()
        self._check(self.lib.he_last_counts(self.h, ctypes.byref(c)), "he_last_counts")
        return {k: int(getattr(c, k)) for k, _ in HeCounts._fields_}

    def prof_select(self, kernel: str | None):
        """Record HIP events around every launch of `kernel` (None stops)."""
        self._check(self.lib.he_prof_select(self.h, (kernel or "").encode()), "he_prof_select")

    def prof_read(self) -> tuple[float, int]:
        """(summed kernel milliseconds, launches) since the last select/read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.he_prof_read(self.h, ctypes.byref(ms), ctypes.byref(n)), "he_prof_read")
        return float(ms.value), int(n.value)

    def prof_read_busy(self) -> tuple[float, float, int]:
        """(summed kernel ms, ms with at least one bracketed launch running, launches)."""
        ms = ctypes.c_double()
        busy = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.he_prof_read_busy(self.h, ctypes.byref(ms), ctypes.byref(busy), ctypes.byref(n)),
                    "he_prof_read_busy")
        return float(ms.value), float(busy.value), int(n.value)

    # ---- transforms ----------------------------------------------------------
    def ntt(self, polys: torch.Tensor, first_mod: int = 0):
        n_limbs = polys.shape[-2]
        n_polys = polys.numel() // (n_limbs * self.n)
        self._check(self.lib.he_ntt(self.h, _ptr(polys), n_polys, n_limbs, first_mod, _stream()), "he_ntt")

    def intt(self, polys: torch.Tensor, first_mod: int = 0):
        n_limbs = polys.shape[-2]
        n_polys = polys.numel() // (n_limbs * self.n)
        self._check(self.lib.he_intt(self.h, _ptr(polys), n_polys, n_limbs, first_mod, _stream()), "he_intt")

    # ---- elementwise -----------------------------------------------------------
    def add(self, out: torch.Tensor, a: Ct, b: Ct) -> Ct:
        level = a.level
        count = a.data.numel() // (2 * level * self.n)
        self._check(self.lib.he_add(self.h, _ptr(out), _ptr(a.data), _ptr(b.data), count, level, float(a.scale),
                                    float(b.scale), _stream()), "he_add")
        return Ct(out, a.scale)

    def hma_plain(self, acc: torch.Tensor, cts: Ct, pts: torch.Tensor, pt_stride: int, pt_scale: float,
                  galois=None, acc_scale: float | None = None) -> Ct:
        """acc (+)= sum_i cts[i] * sigma_{g_i}(pts[i * pt_stride]); accumulates when
        acc_scale (the accumulator's scale) is given."""
        level = acc.shape[-2]
        k = cts.data.numel() // (2 * level * self.n)
        pt_limbs = pts.shape[-2]
        gal = None
        if galois is not None:
            gal = (ctypes.c_int32 * k)(*[int(g) for g in galois])
        io = ctypes.c_double(acc_scale if acc_scale is not None else 0.0)
        self._check(self.lib.he_hma_plain(self.h, _ptr(acc), _ptr(cts.data), k, _ptr(pts), pt_stride, pt_limbs, gal,
                                          level, int(acc_scale is not None), float(cts.scale), float(pt_scale),
                                          ctypes.byref(io), _stream()), "he_hma_plain")
        return Ct(acc, io.value)

    def hma_scalar(self, acc: torch.Tensor, cts: Ct, weights, w_scale: float = 1.0,
                   acc_scale: float | None = None) -> Ct:
        level = acc.shape[-2]
        k = len(weights)
        w = (ctypes.c_int64 * k)(*[int(x) for x in weights])
        io = ctypes.c_double(acc_scale if acc_scale is not None else 0.0)
        self._check(self.lib.he_hma_scalar(self.h, _ptr(acc), _ptr(cts.data), k, w, level,
                                           int(acc_scale is not None), float(cts.scale), float(w_scale),
                                           ctypes.byref(io), _stream()), "he_hma_scalar")
        return Ct(acc, io.value)

    def rescale(self, ct: Ct) -> Ct:
        level = ct.level
        count = ct.data.numel() // (2 * level * self.n)
        out = torch.empty(ct.data.shape[:-2] + (level - 1, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_rescale(self.h, _ptr(out), _ptr(ct.data), count, level, _stream()), "he_rescale")
        return Ct(out, ct.scale / self.q[level - 1])

    # ---- keys / client -----------------------------------------------------------
    def keygen_switch(self, galois: int, s_ntt: torch.Tensor, a: torch.Tensor, e: torch.Tensor,
                      out: torch.Tensor | None = None) -> torch.Tensor:
        """Client side: the switching key of `galois` (0: relinearisation) in the
        exchange layout [L][2][L+1][N]; nothing is stored in the context."""
        if out is None:
            out = torch.empty((self.L, 2, self.L + 1, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_keygen_switch(self.h, int(galois), _ptr(s_ntt), _ptr(a), _ptr(e), _ptr(out),
                                              _stream()), "he_keygen_switch")
        return out

    def upload_keys(self, galois, keys):
        """Server side: store client-made keys ([n][L][2][L+1][N], a device
        tensor or a host uint64 array) for the Galois elements `galois`."""
        galois = [int(g) for g in galois]
        arr = (ctypes.c_int32 * len(galois))(*galois)
        if isinstance(keys, torch.Tensor):
            keys = keys.contiguous()
            self._check(self.lib.he_keys_upload(self.h, arr, len(galois), _ptr(keys), 1, _stream()),
                        "he_keys_upload")
        else:
            host = np.ascontiguousarray(keys, dtype=np.uint64)
            self._check(self.lib.he_keys_upload(self.h, arr, len(galois), host.ctypes.data_as(ctypes.c_void_p), 0,
                                                _stream()), "he_keys_upload")

    def has_key(self, galois: int) -> bool:
        return bool(self.lib.he_has_key(self.h, int(galois)))

    def drop_keys(self, galois=None):
        """Free the keys of `galois` (None: all of them)."""
        if galois is None:
            self._check(self.lib.he_keys_free(self.h, None, 0), "he_keys_free")
        else:
            galois = [int(g) for g in galois]
            arr = (ctypes.c_int32 * len(galois))(*galois)
            self._check(self.lib.he_keys_free(self.h, arr, len(galois)), "he_keys_free")

    def set_workspace(self, buf: torch.Tensor | None):
        """Use a caller-owned device buffer as the workspace (None detaches it);
        the caller keeps `buf` alive while the context uses it."""
        if buf is None:
            self._check(self.lib.he_ctx_set_workspace(self.h, None, 0), "he_ctx_set_workspace")
        else:
            self._check(self.lib.he_ctx_set_workspace(self.h, _ptr(buf), buf.numel() * buf.element_size()),
                        "he_ctx_set_workspace")

    def from_signed(self, coeffs: torch.Tensor, n_limbs: int, first_mod: int = 0) -> torch.Tensor:
        out = torch.empty((n_limbs, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_from_signed(self.h, _ptr(out), _ptr(coeffs), n_limbs, first_mod, _stream()),
                    "he_from_signed")
        return out

    def encrypt_sk(self, pt: torch.Tensor, a: torch.Tensor, e: torch.Tensor, s_ntt: torch.Tensor) -> torch.Tensor:
        level = pt.shape[-2]
        ct = torch.empty((2, level, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_encrypt_sk(self.h, _ptr(ct), _ptr(pt), _ptr(a), _ptr(e), _ptr(s_ntt), level,
                                           _stream()), "he_encrypt_sk")
        return ct

    def decrypt(self, ct: torch.Tensor, s_ntt: torch.Tensor) -> torch.Tensor:
        level = ct.shape[-2]
        out = torch.empty((level, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_decrypt(self.h, _ptr(out), _ptr(ct), _ptr(s_ntt), level, _stream()), "he_decrypt")
        return out

    def encode_coeffs(self, z, scale: float) -> np.ndarray:
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        out = np.empty(self.n, dtype=np.int64)
        rc = self.lib.he_encode_coeffs(self.n, z.ctypes.data_as(_lib.DP), len(z), float(scale),
                                       out.ctypes.data_as(_lib.I64P))
        if rc != 0:
            raise HEError("he_encode_coeffs failed (value too large for the scale?)")
        return out

    def decode_coeffs(self, m, n_values: int) -> np.ndarray:
        m = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
        out = np.empty(n_values, dtype=np.float64)
        rc = self.lib.he_decode_coeffs(self.n, m.ctypes.data_as(_lib.DP), n_values, out.ctypes.data_as(_lib.DP))
        if rc != 0:
            raise HEError("he_decode_coeffs failed")
        return out

    # ---- rotations / square --------------------------------------------------------
    def rotate(self, ct: Ct, k: int, out: torch.Tensor | None = None) -> Ct:
        level = ct.level
        count = ct.data.numel() // (2 * level * self.n)
        out = torch.empty_like(ct.data) if out is None else out
        self._check(self.lib.he_rotate(self.h, _ptr(out), _ptr(ct.data), count, level, int(k), _stream()),
                    "he_rotate")
        return Ct(out, ct.scale)

    def rotate_hoisted(self, ct: Ct, steps) -> Ct:
        level = ct.level
        m = len(steps)
        arr = (ctypes.c_int32 * m)(*[int(k) for k in steps])
        out = torch.empty((m, 2, level, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_rotate_hoisted(self.h, _ptr(ct.data), level, arr, m, _ptr(out), _stream()),
                    "he_rotate_hoisted")
        return Ct(out, ct.scale)

    def rotate_hoisted_batch(self, cts: torch.Tensor, steps, out: torch.Tensor | None = None) -> torch.Tensor:
        """cts [count][2][level][N] -> [count][len(steps)][2][level][N]: each
        ciphertext rotated by every step, one decomposition per ciphertext."""
        level = cts.shape[-2]
        count = cts.numel() // (2 * level * self.n)
        m = len(steps)
        arr = (ctypes.c_int32 * m)(*[int(k) for k in steps])
        if out is None:
            out = torch.empty((count, m, 2, level, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_rotate_hoisted_batch(self.h, _ptr(cts), count, level, arr, m, _ptr(out), _stream()),
                    "he_rotate_hoisted_batch")
        return out

    def rotsum(self, ct: Ct, r_steps: int):
        level = ct.level
        count = ct.data.numel() // (2 * level * self.n)
        self._check(self.lib.he_rotsum(self.h, _ptr(ct.data), count, level, int(r_steps), _stream()), "he_rotsum")

    # ---- batched (ragged) calls --------------------------------------------------
    @staticmethod
    def _ptrs(tensors):
        arr = (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])
        for t in tensors:
            if not (t.is_cuda and t.is_contiguous()):
                raise HEError("batched calls take contiguous device tensors")
        return arr

    def batch_rotate(self, outs, ins, steps, accumulate: bool = False):
        """outs[b] = Rot(ins[b], steps[b]) (or ins[b] + Rot(...)), every item its own level."""
        k = len(ins)
        levels = (ctypes.c_int32 * k)(*[t.shape[-2] for t in ins])
        st = (ctypes.c_int32 * k)(*[int(x) for x in steps])
        self._check(self.lib.he_batch_rotate(self.h, self._ptrs(outs), self._ptrs(ins), levels, st, k,
                                             int(accumulate), _stream()), "he_batch_rotate")

    def batch_rescale(self, outs, ins):
        k = len(ins)
        levels = (ctypes.c_int32 * k)(*[t.shape[-2] for t in ins])
        self._check(self.lib.he_batch_rescale(self.h, self._ptrs(outs), self._ptrs(ins), levels, k, _stream()),
                    "he_batch_rescale")

    def batch_mul_plain(self, outs, cts, pts):
        k = len(cts)
        levels = (ctypes.c_int32 * k)(*[t.shape[-2] for t in cts])
        self._check(self.lib.he_batch_mul_plain(self.h, self._ptrs(outs), self._ptrs(cts), self._ptrs(pts), levels,
                                                k, _stream()), "he_batch_mul_plain")

    def combine_cp_dp(self, z: Ct, spatial: int, per_dense: int) -> Ct:
        o_c, _, level, n = z.data.shape
        n_dense = -(-o_c // per_dense)
        out = torch.empty((n_dense, 2, level, n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_combine_cp_dp(self.h, _ptr(z.data), o_c, level, spatial, per_dense, _ptr(out),
                                              _stream()), "he_combine_cp_dp")
        return Ct(out, z.scale)

    def square(self, ct: Ct) -> Ct:
        level = ct.level
        count = ct.data.numel() // (2 * level * self.n)
        out = torch.empty_like(ct.data)
        self._check(self.lib.he_square(self.h, _ptr(out), _ptr(ct.data), count, level, _stream()), "he_square")
        return Ct(out, ct.scale * ct.scale)

    # ---- layers ----------------------------------------------------------------------
    @staticmethod
    def conv_desc(h, w, c_in, d, stride, pad, o_c, r_steps) -> HeConvDesc:
        desc = HeConvDesc()
        for k, v in dict(h=h, w=w, c_in=c_in, d=d, stride=stride, pad=pad, o_c=o_c, r_steps=r_steps).items():
            setattr(desc, k, int(v))
        return desc

    def conv_densepack(self, x: Ct, desc: HeConvDesc, filt: torch.Tensor, pt_scale: float,
                       out: torch.Tensor | None = None) -> Ct:
        level = x.level
        oh = (desc.h + 2 * desc.pad - desc.d) // desc.stride + 1
        ow = (desc.w + 2 * desc.pad - desc.d) // desc.stride + 1
        total = oh * ow * desc.o_c
        if out is None:
            out = torch.empty((total, 2, level - 1, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_conv_densepack(self.h, _ptr(x.data), level, ctypes.byref(desc), _ptr(filt),
                                               _ptr(out), _stream()), "he_conv_densepack")
        return Ct(out, x.scale * pt_scale / self.q[level - 1])

    def conv_densepack_batch(self, xs: torch.Tensor, scale: float, desc: HeConvDesc, filt: torch.Tensor,
                             pt_scale: float, shared_filters: bool = True, out: torch.Tensor | None = None) -> Ct:
        """DensePack layer on xs[l] (each [M][2][level][N] or [2][level][N]) for every l, one batch.
        filt: one filter set (shared_filters) or one per input stacked on dim 0."""
        n_layers = xs.shape[0]
        level = xs.shape[-2]
        oh = (desc.h + 2 * desc.pad - desc.d) // desc.stride + 1
        ow = (desc.w + 2 * desc.pad - desc.d) // desc.stride + 1
        total = oh * ow * desc.o_c
        if out is None:
            out = torch.empty((n_layers, total, 2, level - 1, self.n), dtype=torch.int64, device="cuda")
        f_stride = 0 if shared_filters else filt[0].numel()
        self._check(self.lib.he_conv_densepack_batch(self.h, n_layers, _ptr(xs), xs[0].numel(), level,
                                                     ctypes.byref(desc), _ptr(filt), f_stride, _ptr(out), _stream()),
                    "he_conv_densepack_batch")
        return Ct(out, scale * pt_scale / self.q[level - 1])

    def combine_cp_dp_batch(self, z: Ct, spatial: int, per_dense: int) -> Ct:
        """z.data [count][o_c][2][level][N] -> [count][n_dense][2][level][N]."""
        count, o_c, _, level, n = z.data.shape
        n_dense = -(-o_c // per_dense)
        out = torch.empty((count, n_dense, 2, level, n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_combine_cp_dp_batch(self.h, count, _ptr(z.data), o_c, level, spatial, per_dense,
                                                    _ptr(out), _stream()), "he_combine_cp_dp_batch")
        return Ct(out, z.scale)

    def gather_onehot(self, y: Ct, k: int, mask: torch.Tensor, mask_scale: float) -> Ct:
        """y.data [count*k][2][level][N] -> [count][2][level][N]: item j of each group to slot j."""
        level = y.level
        count = y.data.numel() // (k * 2 * level * self.n)
        out = torch.empty((count, 2, level, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_gather_onehot(self.h, count, _ptr(y.data), k, _ptr(mask), level, _ptr(out),
                                              _stream()), "he_gather_onehot")
        return Ct(out, y.scale * mask_scale)

    def conv_convpack(self, x: Ct, w: np.ndarray, target_scale: float) -> Ct:
        level = x.level
        k, o_c = w.shape
        wf = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        out = torch.empty((o_c, 2, level - 1, self.n), dtype=torch.int64, device="cuda")
        out_scale = ctypes.c_double(0.0)
        self._check(self.lib.he_conv_convpack(self.h, _ptr(x.data), k, level, wf.ctypes.data_as(_lib.DP), o_c,
                                              float(x.scale), float(target_scale), _ptr(out),
                                              ctypes.byref(out_scale), _stream()), "he_conv_convpack")
        return Ct(out, out_scale.value)

    # ---- tap-style DensePack (hoisted tap rotations) ---------------------------
    def tap_workspace_need(self, n_batch: int, level: int, desc: HeConvDesc, o_c2: int = 0,
                           square: bool = False) -> int:
        need = self.lib.he_tap_workspace_need(self.h, n_batch, level, ctypes.byref(desc), o_c2, int(square))
        if need == 0:
            raise HEError("he_tap_workspace_need: bad geometry or level")
        return need

    def conv_tap(self, xs: torch.Tensor, scale: float, desc: HeConvDesc, filt: torch.Tensor, pt_scale: float,
                 filt_p: torch.Tensor | None = None, out: torch.Tensor | None = None) -> Ct:
        """Tap-style DensePack conv of xs [B][M][2][level][N] with plaintexts
        filt [O][M][d^2][limbs][N] (and their residues mod P, filt_p
        [O][M][d^2][N], for one ModDown per output); returns
        [B][O][2][level-1][N]."""
        nb, level = xs.shape[0], xs.shape[-2]
        if out is None:
            out = torch.empty((nb, desc.o_c, 2, level - 1, self.n), dtype=torch.int64, device="cuda")
        out_scale = ctypes.c_double(0.0)
        fp = None if filt_p is None else _ptr(filt_p)
        self._check(self.lib.he_conv_tap(self.h, nb, _ptr(xs), level, ctypes.byref(desc), _ptr(filt), filt.shape[-2],
                                         fp, float(scale), float(pt_scale), _ptr(out), ctypes.byref(out_scale),
                                         _stream()), "he_conv_tap")
        return Ct(out, out_scale.value)

    def ffconv_layer_tap(self, xs: torch.Tensor, scale: float, desc: HeConvDesc, w1_filt: torch.Tensor,
                         w1_scale: float, mask: torch.Tensor, mask_scale: float, w2: np.ndarray, k_bits: int,
                         square: bool = False, w1_p: torch.Tensor | None = None,
                         out: torch.Tensor | None = None, w2_tab: torch.Tensor | None = None) -> Ct:
        """Tap-style FFConv of xs [B][M][2][level][N]: W1 plaintexts
        [r][M][d^2][limbs][N] (desc.o_c = r; w1_p their residues mod P for
        one ModDown per output), output mask E, W2 (r x o_c2; with w2_tab,
        its int_weight_table at level - 1, the call copies nothing from the
        host and can be captured); returns
        [B][o_c2][2][level-2 (-1 with square)][N]."""
        nb, level = xs.shape[0], xs.shape[-2]
        w2f = np.ascontiguousarray(np.asarray(w2, dtype=np.float64))
        o_c2 = w2f.shape[1]
        h_w2 = None if w2_tab is not None else w2f.ctypes.data_as(_lib.DP)
        lvl_out = level - 2 - (1 if square else 0)
        if out is None:
            out = torch.empty((nb, o_c2, 2, lvl_out, self.n), dtype=torch.int64, device="cuda")
        out_scale = ctypes.c_double(0.0)
        self._check(self.lib.ffconv_layer_tap(self.h, nb, _ptr(xs), level, ctypes.byref(desc), _ptr(w1_filt),
                                              w1_filt.shape[-2], None if w1_p is None else _ptr(w1_p),
                                              float(scale), float(w1_scale), _ptr(mask),
                                              float(mask_scale), h_w2, None if w2_tab is None else _ptr(w2_tab),
                                              o_c2, int(k_bits),
                                              int(square), _ptr(out), ctypes.byref(out_scale), _stream()),
                    "ffconv_layer_tap")
        return Ct(out, out_scale.value)

    def him2col_workspace_need(self, n_batch: int, level: int, desc: HeConvDesc) -> int:
        need = self.lib.he_him2col_workspace_need(self.h, n_batch, level, ctypes.byref(desc))
        if need == 0:
            raise HEError("he_him2col_workspace_need: bad geometry or level")
        return need

    def him2col(self, xs: torch.Tensor, scale: float, desc: HeConvDesc, masks: torch.Tensor, mask_scale: float,
                out: torch.Tensor | None = None) -> Ct:
        """Homomorphic Im2Col of DensePack inputs xs [B][M][2][level][N]
        with the tap masks [d^2][limbs][N]; returns [B][K][2][level-1][N]."""
        nb, level = xs.shape[0], xs.shape[-2]
        k = desc.d * desc.d * desc.c_in
        if out is None:
            out = torch.empty((nb, k, 2, level - 1, self.n), dtype=torch.int64, device="cuda")
        out_scale = ctypes.c_double(0.0)
        self._check(self.lib.he_him2col(self.h, nb, _ptr(xs), level, ctypes.byref(desc), _ptr(masks),
                                        masks.shape[-2], float(scale), float(mask_scale), _ptr(out),
                                        ctypes.byref(out_scale), _stream()), "he_him2col")
        return Ct(out, out_scale.value)

    # ---- layer pieces for iteration-level batching ------------------------------
    def densepack_hma(self, xs: torch.Tensor, desc: HeConvDesc, filt: torch.Tensor, shared_filters: bool = True,
                      out: torch.Tensor | None = None) -> torch.Tensor:
        """MulPC part of a DensePack layer on xs[l] ([B][M][2][level][N]):
        returns the unsummed accumulators [B * o_c * S][2][level][N]."""
        n_layers = xs.shape[0]
        level = xs.shape[-2]
        oh = (desc.h + 2 * desc.pad - desc.d) // desc.stride + 1
        ow = (desc.w + 2 * desc.pad - desc.d) // desc.stride + 1
        total = n_layers * oh * ow * desc.o_c
        if out is None:
            out = torch.empty((total, 2, level, self.n), dtype=torch.int64, device="cuda")
        f_stride = 0 if shared_filters else filt[0].numel()
        self._check(self.lib.he_densepack_hma(self.h, n_layers, _ptr(xs), xs[0].numel(), level, ctypes.byref(desc),
                                              _ptr(filt), f_stride, _ptr(out), _stream()), "he_densepack_hma")
        return out

    def rotsum_groups(self, groups):
        """One rotate-and-add step for each (acc tensor [count][2][level][N], step)."""
        arr = (_lib.HeRotsumGroup * len(groups))()
        for i, (acc, step) in enumerate(groups):
            if not (acc.is_cuda and acc.is_contiguous()):
                raise HEError("rotsum_groups takes contiguous device tensors")
            arr[i].acc = acc.data_ptr()
            arr[i].level = acc.shape[-2]
            arr[i].count = acc.numel() // (2 * acc.shape[-2] * self.n)
            arr[i].step = int(step)
        self._check(self.lib.he_rotsum_groups(self.h, arr, len(groups), _stream()), "he_rotsum_groups")

    def ffconv_tail_batch(self, acc: torch.Tensor, n_layers: int, desc: HeConvDesc, mask: torch.Tensor,
                          w2_tabs: torch.Tensor, o_c2: int, square: bool, out: torch.Tensor | None = None):
        """Rescale + gather + 1x1 ConvPack (+ x^2) of summed W1 accumulators
        acc [n_layers * r * S][2][level][N]; returns [n_layers][o_c2][2][..][N]."""
        level = acc.shape[-2]
        lvl_out = level - 2 - (1 if square else 0)
        if out is None:
            out = torch.empty((n_layers, o_c2, 2, lvl_out, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.ffconv_tail_batch(self.h, n_layers, _ptr(acc), level, ctypes.byref(desc), _ptr(mask),
                                               _ptr(w2_tabs), o_c2, int(square), _ptr(out), _stream()),
                    "ffconv_tail_batch")
        return out

    def ffconv_layer_convpack(self, x: Ct, w1: np.ndarray, w2: np.ndarray, target_scale: float,
                              square: bool = False) -> Ct:
        """FFConv with both factors under ConvPack on the K Im2Col ciphertexts
        x ([K][2][level][N]); w1: K x r (Eq. 1 rows), w2: r x o_c."""
        level = x.level
        k, r = w1.shape
        o_c = w2.shape[1]
        w1f = np.ascontiguousarray(np.asarray(w1, dtype=np.float64))
        w2f = np.ascontiguousarray(np.asarray(w2, dtype=np.float64))
        lvl_out = level - 2 - (1 if square else 0)
        out = torch.empty((o_c, 2, lvl_out, self.n), dtype=torch.int64, device="cuda")
        out_scale = ctypes.c_double(0.0)
        self._check(self.lib.ffconv_layer_convpack(self.h, _ptr(x.data), k, level, w1f.ctypes.data_as(_lib.DP), r,
                                                   w2f.ctypes.data_as(_lib.DP), o_c, float(x.scale),
                                                   float(target_scale), int(square), _ptr(out),
                                                   ctypes.byref(out_scale), _stream()), "ffconv_layer_convpack")
        return Ct(out, out_scale.value)

    def ffconv_layer(self, x: Ct, desc: HeConvDesc, w1_filt: torch.Tensor, w1_pt_scale: float,
                     mask: torch.Tensor, mask_scale: float, w2: np.ndarray, k_bits: int, square: bool,
                     out: torch.Tensor | None = None) -> Ct:
        level = x.level
        r, o_c2 = w2.shape
        wf = np.ascontiguousarray(np.asarray(w2, dtype=np.float64))
        lvl_out = level - 2 - (1 if square else 0)
        if out is None:
            out = torch.empty((o_c2, 2, lvl_out, self.n), dtype=torch.int64, device="cuda")
        self._check(self.lib.ffconv_layer(self.h, _ptr(x.data), level, ctypes.byref(desc), _ptr(w1_filt),
                                          _ptr(mask), wf.ctypes.data_as(_lib.DP), o_c2, int(k_bits), int(square),
                                          _ptr(out), _stream()), "ffconv_layer")
        y_scale = x.scale * w1_pt_scale / self.q[level - 1]
        z_scale = y_scale * mask_scale * 2.0**k_bits / self.q[level - 2]
        if square:
            z_scale = z_scale * z_scale / self.q[level - 3]
        return Ct(out, z_scale)

    def int_weight_table(self, w: np.ndarray, k_bits: int, level: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """Device table of round(w * 2^k_bits) (row-major w) for limbs < level."""
        wf = np.ascontiguousarray(np.asarray(w, dtype=np.float64).ravel())
        if out is None:
            out = torch.empty((2 * wf.size * level,), dtype=torch.int64, device="cuda")
        self._check(self.lib.he_int_weight_table(self.h, wf.ctypes.data_as(_lib.DP), wf.size, int(k_bits), level,
                                                 _ptr(out), _stream()), "he_int_weight_table")
        return out

    def ffconv_workspace_need(self, n_layers: int, level: int, desc: HeConvDesc, o_c2: int, square: bool) -> int:
        return int(self.lib.he_ffconv_workspace_need(self.h, n_layers, level, ctypes.byref(desc), o_c2,
                                                      int(square)))

    def ffconv_layer_batch(self, xs: torch.Tensor, scale: float, desc: HeConvDesc, w1_filts: torch.Tensor,
                           w1_pt_scale: float, mask: torch.Tensor, mask_scale: float, w2_tabs: torch.Tensor,
                           o_c2: int, k_bits: int, square: bool, out: torch.Tensor | None = None,
                           shared_w1: bool = False) -> Ct:
        """len(xs) independent FFConv layers (inputs xs[l], all at `scale`, with
        filters w1_filts[l] -- or one filter set for all when shared_w1 -- and
        W2 tables w2_tabs[l]) in one call."""
        n_layers = xs.shape[0]
        level = xs.shape[-2]
        assert shared_w1 or w1_filts.shape[0] == n_layers
        assert w2_tabs.shape[0] == n_layers
        assert xs.is_contiguous() and w1_filts.is_contiguous() and w2_tabs.is_contiguous()
        lvl_out = level - 2 - (1 if square else 0)
        if out is None:
            out = torch.empty((n_layers, o_c2, 2, lvl_out, self.n), dtype=torch.int64, device="cuda")
        in_stride = xs[0].numel()
        f_stride = 0 if shared_w1 else w1_filts[0].numel()
        self._check(self.lib.ffconv_layer_batch(self.h, n_layers, _ptr(xs), in_stride, level, ctypes.byref(desc),
                                                _ptr(w1_filts), f_stride, _ptr(mask), _ptr(w2_tabs), o_c2,
                                                int(square), _ptr(out), _stream()), "ffconv_layer_batch")
        y_scale = scale * w1_pt_scale / self.q[level - 1]
        z_scale = y_scale * mask_scale * 2.0**k_bits / self.q[level - 2]
        if square:
            z_scale = z_scale * z_scale / self.q[level - 3]
        return Ct(out, z_scale)

    def capture(self, fn):
        """Records the library calls fn() makes into a HIP graph (on a side
        stream) and returns (Graph, fn's result).  fn must allocate nothing:
        pass preallocated outputs."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = ctypes.c_void_p()
        with torch.cuda.stream(side):
            self._check(self.lib.he_graph_begin(self.h, _stream()), "he_graph_begin")
            try:
                res = fn()
            except BaseException:
                if self.lib.he_graph_end(self.h, _stream(), ctypes.byref(g)) == 0 and g:
                    self.lib.he_graph_destroy(g)
                raise
            self._check(self.lib.he_graph_end(self.h, _stream(), ctypes.byref(g)), "he_graph_end")
        torch.cuda.current_stream().wait_stream(side)
        return Graph(self, g), res
