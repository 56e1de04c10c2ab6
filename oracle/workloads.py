"""Client set-up for the evaluated workloads (test infrastructure; see package doc).

Builds the oracle's key material from the `synth` draws: the secret, one
rotation key per Galois element (stream index = the element), the
relinearisation key (stream index 0) and secret-key encryptions.
"""
from __future__ import annotations

import synth

from . import params as P
from . import scheme
from .encoding import encode
from .ring import galois_for_rotation


def make_context(params, workload, rotations=(), relin=False, secret_index=0):
    ctx = scheme.Context(params, synth.ternary_secret(workload, params.n, secret_index))
    moduli = params.q + [params.p]
    done = set()
    for k in rotations:
        g = galois_for_rotation(k, params.n)
        if g in done or g == 1:
            continue
        done.add(g)
        a, e = synth.switch_key_draws(workload, g, moduli, params.n, params.max_level)
        ctx.add_rotation_key(k, a, e)
    if relin:
        a, e = synth.switch_key_draws(workload, synth.RELIN_INDEX, moduli, params.n, params.max_level)
        ctx.set_relin_key(a, e)
    return ctx


def encrypt_slots(ctx, slots_values, level, scale, workload, index):
    p = ctx.params
    pt = encode(slots_values, p, level, scale)
    a, e = synth.encryption_draws(workload, index, p.q[:level], p.n)
    return ctx.encrypt(pt, scale, a, e)


PARAMS = {
    "plain_n4096": P.plain_n4096,
    "ffconv_n8192": P.ffconv_n8192,
    "cifar_n16384": P.cifar_n16384,
}
