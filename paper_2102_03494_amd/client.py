"""Client side of the protocol (the party that holds the secret key).

In the paper's setting (Section 1; Section 3, MLaaS scenario) the client
encrypts its image, the server evaluates the network with plaintext weights
and the client decrypts the prediction.  This module generates the secret and
the switching keys from the seeded draws of ``synth``, encodes and encrypts
slot vectors and decrypts results, calling the library for every ring
operation (encoding's FFT and the CRT of decryption run on the host).

The client works in a library context of its own.  The server's context
never sees the secret: it receives only the switching keys, through
``he_keys_upload`` in the exchange layout, and the ciphertexts.
"""
from __future__ import annotations

import numpy as np
import torch

import synth

from .he import Ct, HEContext, galois_for_rotation, to_device, to_host


class Client:
    def __init__(self, server: HEContext, workload, secret_index: int = 0):
        """`server` is the evaluating party's context: it only ever receives keys."""
        self.server = server
        self.ctx = HEContext(server.n, server.q_bits, server.p_bits, workspace_bytes=16 << 20, tuned=False)
        ctx = self.ctx
        self.workload = workload
        n, big_l = ctx.n, ctx.L
        s = synth.ternary_secret(workload, n, secret_index)
        self.s_coeff = torch.from_numpy(s).cuda()
        s_ntt = ctx.from_signed(self.s_coeff, big_l + 1, 0)
        ctx.ntt(s_ntt.view(1, big_l + 1, n))
        self.s_ntt = s_ntt

    # ---- keys ------------------------------------------------------------------
    def switch_key(self, key_index: int) -> torch.Tensor:
        """The key for Galois element key_index (0: relinearisation), exchange
        layout [L][2][L+1][N], made in the client's own context."""
        c = self.ctx
        a, e = synth.switch_key_draws(self.workload, key_index, c.moduli, c.n, c.L)
        return c.keygen_switch(key_index, self.s_ntt, to_device(a), torch.from_numpy(e).cuda())

    def _send(self, key_index: int, server: HEContext | None):
        server = self.server if server is None else server
        if not server.has_key(key_index):
            key = self.switch_key(key_index)
            server.upload_keys([key_index], key.view(1, *key.shape))
            del key

    def gen_rotation_keys(self, steps, server: HEContext | None = None):
        """Make the rotation keys of `steps` and upload them to the server."""
        for k in steps:
            g = galois_for_rotation(int(k), self.ctx.n)
            if g != 1:
                self._send(g, server)

    def gen_relin_key(self, server: HEContext | None = None):
        self._send(synth.RELIN_INDEX, server)

    # ---- plaintexts -----------------------------------------------------------------
    def encode(self, z, level: int, scale: float) -> torch.Tensor:
        """NTT-domain plaintext [level][N] of real slot values z."""
        from .layers import PlainEncoder
        return PlainEncoder(self.ctx).encode(z, level, scale)

    def encrypt_pt(self, pt: torch.Tensor, scale: float, index: int) -> Ct:
        c = self.ctx
        level = pt.shape[-2]
        a, e = synth.encryption_draws(self.workload, index, c.q[:level], c.n)
        ct = c.encrypt_sk(pt, to_device(a), torch.from_numpy(e).cuda(), self.s_ntt)
        return Ct(ct.view(1, 2, level, c.n), scale)

    def encrypt(self, z, level: int, scale: float, index: int) -> Ct:
        return self.encrypt_pt(self.encode(z, level, scale), scale, index)

    # ---- decryption -----------------------------------------------------------------
    def decrypt_coeffs(self, ct_one: torch.Tensor) -> list[int]:
        """Centred integer coefficients of c0 + c1*s (exact CRT over the limbs)."""
        c = self.ctx
        m = c.decrypt(ct_one.contiguous(), self.s_ntt)
        level = m.shape[0]
        c.intt(m.view(1, level, c.n))
        limbs = to_host(m)
        moduli = c.q[:level]
        big_q = 1
        for q in moduli:
            big_q *= q
        parts = []
        for t, q in enumerate(moduli):
            qhat = big_q // q
            parts.append((qhat, pow(qhat % q, -1, q), q, limbs[t]))
        out = []
        for k in range(c.n):
            x = 0
            for qhat, qinv, q, col in parts:
                x += (int(col[k]) * qinv % q) * qhat
            x %= big_q
            out.append(x - big_q if x > big_q // 2 else x)
        return out

    def decrypt(self, ct_one: torch.Tensor, scale: float, n_values: int | None = None,
                limbs: int | None = None) -> np.ndarray:
        """Real slot values.  `limbs` keeps only the first limbs (modulus drop),
        valid when |message * scale| < q_0 / 2; with one limb the centring is
        vectorised."""
        n_values = self.ctx.n // 2 if n_values is None else n_values
        if limbs is not None:
            ct_one = ct_one[:, :limbs]
        if ct_one.shape[-2] == 1:
            c = self.ctx
            m = c.decrypt(ct_one.contiguous(), self.s_ntt)
            c.intt(m.view(1, 1, c.n))
            v = to_host(m)[0].astype(np.int64)
            q = c.q[0]
            v = np.where(v > q // 2, v - q, v).astype(np.float64)
            return self.ctx.decode_coeffs(v / scale, n_values)
        coeffs = self.decrypt_coeffs(ct_one)
        m = np.array([float(x) for x in coeffs]) / scale
        return self.ctx.decode_coeffs(m, n_values)
