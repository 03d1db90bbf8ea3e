"""The C-ABI library loads and exports every symbol its header declares (CPU only:
no call here touches a GPU; only host-side argument checks are exercised)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lob.h")
LIB = os.path.join(ROOT, "paper_2511_02136_amd", "liblob.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ \*]*?\b(lob_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("lob_init", "lob_reset", "lob_step", "lob_rollout", "lob_observe", "lob_export_books",
              "lob_export_state", "lob_destroy", "lob_strerror"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_host_side_argument_checks():
    lib = ctypes.CDLL(LIB)
    lib.lob_strerror.restype = ctypes.c_char_p
    assert lib.lob_strerror(0) == b"ok"
    assert lib.lob_strerror(-1) == b"invalid argument"
    assert lib.lob_strerror(-4).startswith(b"call out of order")
    # NULL arguments are rejected before any device call
    lib.lob_init.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lob_init(None, None) == -1
    lib.lob_step.argtypes = [ctypes.c_void_p] * 5
    assert lib.lob_step(None, None, None, None, None) == -1
    lib.lob_rollout.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lob_rollout(None, None, 1, None, None, None) == -1
    lib.lob_destroy.argtypes = [ctypes.c_void_p]
    assert lib.lob_destroy(None) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_host_side_checks_of_the_actor_critic():
    """Argument checks of the actor-critic entry points, all taken before any device call
    (the pointers passed where a check must fail first are never dereferenced), and the
    workspace size of the fused PPO call: 256 workgroup partials at most, plus one partial
    per 64 of them for the first reduction level, of 78,864 floats each (78,858 parameters,
    4 loss sums, 2 of padding), plus room for an aligned copy of the parameters and for
    W2 (256 x 256) transposed."""
    lib = ctypes.CDLL(LIB)
    p, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    lib.lob_ppo_workspace_bytes.argtypes = [i32]
    lib.lob_ppo_workspace_bytes.restype = ctypes.c_int64
    pw, copy = 78864 * 4, 78858 * 4 + 16 + 256 * 256 * 4 + 16
    assert lib.lob_ppo_workspace_bytes(0) == -1 and lib.lob_ppo_workspace_bytes(-3) == -1
    assert lib.lob_ppo_workspace_bytes(1) == (1 + 1) * pw + copy
    assert lib.lob_ppo_workspace_bytes(64 * 100 + 1) == (101 + 2) * pw + copy
    assert lib.lob_ppo_workspace_bytes(131072) == (256 + 4) * pw + copy
    assert lib.lob_ppo_workspace_bytes(1 << 30) == (256 + 4) * pw + copy
    lib.lob_ppo_fwd_bwd.argtypes = [p] * 8 + [i32, i32, f32, f32, f32, p, ctypes.c_int64, p, p, p]
    d = [p(0x1000 + 16 * k) for k in range(7)]
    ws, big = p(0x20000), 1 << 40

    def call(m=64, n_act=9, clip=0.2, w=ws, wb=big, ptrs=d):
        # the observation scale (third argument) is optional
        return lib.lob_ppo_fwd_bwd(*ptrs[:2], None, *ptrs[2:], m, n_act, clip, 0.5, 0.01, w, wb, p(0x3000), p(0x4000),
                                   None)
    assert lib.lob_ppo_fwd_bwd(*([None] * 8), 64, 9, 0.2, 0.5, 0.01, None, 0, None, None, None) == -1
    assert call(ptrs=[None] + d[1:]) == -1
    assert call(m=0) == -1 and call(n_act=0) == -1 and call(n_act=10) == -1 and call(clip=0.0) == -1
    assert call(wb=lib.lob_ppo_workspace_bytes(64) - 1) == -1   # too small
    assert call(w=p(0x20004)) == -1                              # not 16-byte aligned
    lib.lob_gae.argtypes = [p, p, p, p, i32, i32, f32, f32, p, p, p]
    assert lib.lob_gae(None, None, None, None, 4, 4, 0.99, 0.95, None, None, None) == -1
    assert lib.lob_gae(*d[:4], 0, 4, 0.99, 0.95, d[4], d[5], None) == -1
    assert lib.lob_gae(*d[:4], 4, 0, 0.99, 0.95, d[4], d[5], None) == -1
    lib.lob_policy_forward.argtypes = [p, p, p, i32, i32, p, ctypes.c_uint64, p, i32, p, p, p, p, p]
    assert lib.lob_policy_forward(None, None, None, 1, 8, None, 0, None, 0, None, None, None, None, None) == -1
    n_act = (i32 * 2)(9, 9)
    assert lib.lob_policy_forward(d[0], d[1], None, 0, 8, n_act, 0, None, 0, None, d[2], d[3], d[4], None) == -1
    assert lib.lob_policy_forward(d[0], d[1], None, 2, 0, n_act, 0, None, 0, None, d[2], d[3], d[4], None) == -1
    bad = (i32 * 2)(9, 10)
    assert lib.lob_policy_forward(d[0], d[1], None, 2, 8, bad, 0, None, 0, None, d[2], d[3], d[4], None) == -1
    lib.lob_counter_bump.argtypes = [p, p]
    assert lib.lob_counter_bump(None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_host_side_checks_of_the_state_import():
    """lob_import_state rejects a NULL context, NULL books and NULL state before any
    device call."""
    lib = ctypes.CDLL(LIB)
    p = ctypes.c_void_p
    lib.lob_import_state.argtypes = [p, p, p, p, p, ctypes.c_int32, p]
    assert lib.lob_import_state(None, None, None, None, None, 0, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_host_side_checks_of_the_noalloc_ppo_call():
    """lob_ppo_fwd_bwd_noalloc rejects NULL pointers and bad sizes before any device call
    (its fixed scratch is resolved only after the checks)."""
    lib = ctypes.CDLL(LIB)
    p, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    lib.lob_ppo_fwd_bwd_noalloc.argtypes = [p, p, p, p, p, p, p, p, i32, i32, f32, f32, f32, p, p, p]
    assert lib.lob_ppo_fwd_bwd_noalloc(None, None, None, None, None, None, None, None, 64, 9, 0.2, 0.5, 0.01,
                                       None, None, None) == -1
    fake = ctypes.c_void_p(16)  # never dereferenced: a size check fails first
    args = [fake, fake, None] + [fake] * 5
    assert lib.lob_ppo_fwd_bwd_noalloc(*args, 0, 9, 0.2, 0.5, 0.01, fake, fake, None) == -1
    assert lib.lob_ppo_fwd_bwd_noalloc(*args, 64, 10, 0.2, 0.5, 0.01, fake, fake, None) == -1
    assert lib.lob_ppo_fwd_bwd_noalloc(*args, 64, 9, 0.0, 0.5, 0.01, fake, fake, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_host_side_checks_of_the_recurrent_actor_critic():
    """Workspace size of the recurrent loss (per sample: hidden state, embedding, input
    gates then their gradients, hidden-gate, embedding and output gradients = 128 + 128 +
    384 + 384 + 128 + 16 floats; one more hidden state per sequence; loss sums per 64
    samples; the weights prepared for 16-byte loads (W_e^T, W_i^T, W_h^T, W_i, W_h, W_o^T
    and W_o padded); weight-gradient partials of 105,612 floats for one workgroup per 64
    samples, at most 256, and the first reduction level's chunk sums) and argument
    checks before any device call."""
    lib = ctypes.CDLL(LIB)
    p, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    lib.lob_gru_ppo_workspace_bytes.argtypes = [i32, i32]
    lib.lob_gru_ppo_workspace_bytes.restype = ctypes.c_int64

    def expect(T, m):
        S = T * m
        nwg = min(256, (S + 63) // 64)
        nch = (nwg + 63) // 64
        weights = 128 * 48 + 4 * 384 * 128 + 2 * 16 * 128  # the sequence kernel's prepared weights
        return 4 * ((T + 1) * m * 128 + S * (128 + 384 + 384 + 128 + 16) + ((S + 63) // 64) * 4 + weights
                    + (nwg + nch) * 105612)
    assert lib.lob_gru_ppo_workspace_bytes(0, 5) == -1 and lib.lob_gru_ppo_workspace_bytes(5, 0) == -1
    for T, m in ((1, 1), (8, 20), (128, 1024)):
        assert lib.lob_gru_ppo_workspace_bytes(T, m) == expect(T, m), (T, m)
    lib.lob_gru_ppo_fwd_bwd.argtypes = [p] * 10 + [i32, i32, i32, f32, f32, f32, p, ctypes.c_int64, p, p, p]
    d = [p(0x1000 + 16 * k) for k in range(10)]
    d[2] = None  # the observation scale is optional

    def call(T=8, m=20, n_act=9, clip=0.2, w=p(0x40000), wb=1 << 40, ptrs=d):
        return lib.lob_gru_ppo_fwd_bwd(*ptrs, T, m, n_act, clip, 0.5, 0.01, w, wb, p(0x3000), p(0x4000), None)
    assert call(ptrs=[None] + d[1:]) == -1
    assert call(T=0) == -1 and call(m=0) == -1 and call(n_act=10) == -1 and call(clip=0.0) == -1
    assert call(wb=lib.lob_gru_ppo_workspace_bytes(8, 20) - 1) == -1
    assert call(w=p(0x40008)) == -1
    lib.lob_gru_step.argtypes = [p] * 6 + [i32, i32, p, ctypes.c_uint64, p, i32, p, p, p, p, p]
    n_act = (i32 * 2)(9, 3)
    assert lib.lob_gru_step(None, *d[1:6], 2, 8, n_act, 0, None, 0, None, d[6], d[7], d[8], None) == -1
    assert lib.lob_gru_step(*d[:6], 0, 8, n_act, 0, None, 0, None, d[6], d[7], d[8], None) == -1
    assert lib.lob_gru_step(*d[:6], 2, 0, n_act, 0, None, 0, None, d[6], d[7], d[8], None) == -1
