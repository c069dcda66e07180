"""CPU-side checks of the C ABI: the library loads, exports every declared entry point,
and validates arguments on the host before anything reaches a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bpstereo.h")
LIB = os.path.join(ROOT, "paper_1709_06509_amd", "libbpstereo.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbpstereo.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["stereo_cost_volume", "bp_hierarchical_solve", "bp_energy", "bp_workspace_bytes", "bp_last_error",
              "stereo_luma", "bp_context_create", "bp_context_destroy"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_validation_without_gpu(lib):
    from paper_1709_06509_amd import bpstereo as B

    L = B.library()
    p = B.make_params(16, 3, [8, 8, 8], 64, 4)
    need = L.bp_workspace_bytes(128, 96, ctypes.byref(p))
    assert need > 4 * 128 * 96 * 16 * 2  # at least the finest scale's four message volumes
    for bad in [B.make_params(0, 3, 8, 64, 4), B.make_params(300, 3, 8, 64, 4), B.make_params(16, 9, 8, 64, 4),
                B.make_params(16, 3, 8, -1, 4), B.make_params(16, 3, 8, 64, -1), B.make_params(16, 3, 2000, 64, 4),
                B.make_params(16, 3, 8, 64, 4, skip_mode=3), B.make_params(16, 3, 8, 64, 4, skip_mode=1, converge_iters=3)]:
        assert L.bp_workspace_bytes(128, 96, ctypes.byref(bad)) == 0
    assert L.bp_workspace_bytes(0, 96, ctypes.byref(p)) == 0
    # invalid calls are rejected before any launch, with a message
    rc = L.bp_hierarchical_solve(None, ctypes.c_void_p(16), 128, 96, ctypes.byref(B.make_params(0, 3, 8, 64, 4)),
                                 ctypes.c_void_p(256), 1 << 30, ctypes.c_void_p(16), None, None, None)
    assert rc == B.BP_E_INVAL and b"num_disp" in L.bp_last_error()
    rc = L.bp_hierarchical_solve(None, ctypes.c_void_p(16), 128, 96, ctypes.byref(p), ctypes.c_void_p(256), need - 1,
                                 ctypes.c_void_p(16), None, None, None)
    assert rc == B.BP_E_WORKSPACE
    rc = L.stereo_cost_volume(ctypes.c_void_p(16), ctypes.c_void_p(16), 64, 64, 16, 4, 256, 1024,
                              ctypes.c_void_p(16), None, None)
    assert rc == B.BP_E_INVAL and b"window" in L.bp_last_error()
    rc = L.bp_energy(ctypes.c_void_p(16), ctypes.c_void_p(16), 8, 8, 4, 1, 1, ctypes.c_void_p(16), ctypes.c_void_p(16),
                     1, None)
    assert rc == B.BP_E_WORKSPACE


def test_workspace_grows_with_shape(lib):
    from paper_1709_06509_amd import bpstereo as B

    L = B.library()
    p = B.make_params(128, 5, 12, 64, 4)
    big = L.bp_workspace_bytes(1920, 1080, ctypes.byref(p))
    # cost pyramid (~4/3 of the finest) + two message buffers (finest and next) + state
    assert 5 * 1920 * 1080 * 128 * 2 < big < 8 * 1920 * 1080 * 128 * 2


def test_jacobi_host_validation(lib):
    from paper_1709_06509_amd import bpstereo as B

    L = B.library()
    need = L.bp_jacobi_workspace_bytes(64, 48, 16)
    assert need >= 8 * 64 * 48 * 16 * 2  # two sets of four message volumes
    for bad in [(0, 48, 16), (64, 0, 16), (64, 48, 0), (64, 48, 257), (16385, 4, 4)]:
        assert L.bp_jacobi_workspace_bytes(*bad) == 0
    p = ctypes.c_void_p
    rc = L.bp_jacobi_iterations(p(16), 64, 48, 16, 64, 4, -1, None, p(16), p(256), need, None)
    assert rc == B.BP_E_INVAL and b"iterations" in L.bp_last_error()
    rc = L.bp_jacobi_iterations(p(16), 64, 48, 16, -1, 4, 2, None, p(16), p(256), need, None)
    assert rc == B.BP_E_INVAL
    rc = L.bp_jacobi_iterations(None, 64, 48, 16, 64, 4, 2, None, p(16), p(256), need, None)
    assert rc == B.BP_E_INVAL
    rc = L.bp_jacobi_iterations(p(16), 64, 48, 16, 64, 4, 2, None, p(16), p(256), need - 1, None)
    assert rc == B.BP_E_WORKSPACE
    rc = L.bp_jacobi_iterations(p(16), 64, 48, 16, 64, 4, 2, None, p(16), p(255), need, None)
    assert rc == B.BP_E_WORKSPACE


def test_noalloc_host_validation(lib):
    """The allocation-free solve checks its arguments and the scratch size on the host: a
    shape whose workspace exceeds the static scratch is refused before any GPU call."""
    from paper_1709_06509_amd import bpstereo as B

    L = B.library()
    cap = L.bp_noalloc_scratch_bytes()
    assert cap == 32 << 20
    prod = B.make_params(16, 4, 10, 64, 4, skip_mode=1)
    assert L.bp_workspace_bytes(384, 288, ctypes.byref(prod)) <= cap
    big = B.make_params(64, 4, 10, 64, 4)
    assert L.bp_workspace_bytes(640, 480, ctypes.byref(big)) > cap
    p = ctypes.c_void_p
    rc = L.bp_hierarchical_solve_noalloc(None, p(16), 640, 480, ctypes.byref(big), p(16), None, None, None)
    assert rc == B.BP_E_WORKSPACE and b"static scratch" in L.bp_last_error()
    rc = L.bp_hierarchical_solve_noalloc(None, p(16), 640, 480, ctypes.byref(B.make_params(0, 4, 10, 64, 4)), p(16),
                                         None, None, None)
    assert rc == B.BP_E_INVAL
    rc = L.bp_hierarchical_solve_noalloc(None, None, 64, 48, ctypes.byref(prod), p(16), None, None, None)
    assert rc == B.BP_E_INVAL


def test_warmstart_solve_host_validation(lib):
    """The one-call warm-started solve rejects bad arguments on the host: NULL pointers, caller
    messages (the network provides the start), a single scale, a disparity count the one-launch
    network does not take, and a short workspace."""
    from paper_1709_06509_amd import bpstereo as B
    from paper_1709_06509_amd import warmstart as WS

    L = WS._lib()
    p = ctypes.c_void_p
    good = B.make_params(64, 4, [6, 4, 4, 0], 64, 4)
    need = L.bp_workspace_bytes(160, 120, ctypes.byref(good))
    args = lambda prm, ws=need, left=p(16), cw=p(16): (None, left, p(16), p(16), 160, 120, ctypes.byref(prm), p(16),
                                                       cw, p(256), ws, p(16), None, None, None)
    rc = L.bp_warmstart_solve(*args(good, left=None))
    assert rc == B.BP_E_INVAL and b"NULL" in L.bp_last_error()
    rc = L.bp_warmstart_solve(*args(good, cw=None))
    assert rc == B.BP_E_INVAL
    warm = B.make_params(64, 4, [6, 4, 4, 0], 64, 4)
    warm.warm_msgs = 4096
    rc = L.bp_warmstart_solve(*args(warm))
    assert rc == B.BP_E_INVAL and b"warm_msgs" in L.bp_last_error()
    rc = L.bp_warmstart_solve(*args(B.make_params(64, 1, [6], 64, 4)))
    assert rc == B.BP_E_INVAL
    for D in (8, 40, 80, 128):
        prm = B.make_params(D, 4, [6, 4, 4, 0], 64, 4)
        rc = L.bp_warmstart_solve(*args(prm, ws=L.bp_workspace_bytes(160, 120, ctypes.byref(prm))))
        assert rc == B.BP_E_UNSUPPORTED and b"multiple of 16" in L.bp_last_error(), D
    rc = L.bp_warmstart_solve(*args(good, ws=need - 1))
    assert rc == B.BP_E_WORKSPACE
    rc = L.bp_warmstart_solve(*args(good, cw=p(24)))  # the network reads its weights 16 bytes at a time
    assert rc == B.BP_E_INVAL and b"16-byte" in L.bp_last_error()


def test_convolution_alignment_validation(lib):
    """The convolution entry points read activations and weights 16 bytes at a time and reject
    operands that are not 16-byte aligned before any device work (the pointers here are never
    dereferenced)."""
    from paper_1709_06509_amd import bpstereo as B
    from paper_1709_06509_amd import warmstart as WS

    L = WS._lib()
    p = ctypes.c_void_p
    rc = L.bp_conv3x3_forward(p(24), 8, 8, 16, p(256), None, 32, 32, 1, None, p(256), None, None)
    assert rc == B.BP_E_INVAL and b"16-byte" in L.bp_last_error()
    rc = L.bp_conv3x3_forward(p(256), 8, 8, 16, p(264), None, 32, 32, 1, None, p(256), None, None)
    assert rc == B.BP_E_INVAL and b"16-byte" in L.bp_last_error()
    rc = L.bp_conv3x3_data_grad(p(24), 8, 8, 32, p(256), 16, 32, None, p(256), p(256), None, None)
    assert rc == B.BP_E_INVAL and b"16-byte" in L.bp_last_error()
    ws = L.bp_cnn_workspace_bytes(8, 8, 16)
    assert ws > 0
    rc = L.bp_cnn_forward(p(24), 8, 8, 16, p(256), p(256), p(256), ws, p(256), None)
    assert rc == B.BP_E_INVAL and b"16-byte" in L.bp_last_error()
    rc = L.bp_cnn_forward(p(256), 8, 8, 16, p(256), p(264), p(256), ws, p(256), None)
    assert rc == B.BP_E_INVAL and b"16-byte" in L.bp_last_error()


def test_batch_message_bits(lib):
    """The batch's message storage: 12 bits wherever lambda T <= 4095 (any num_disp), else
    16; 0 for a batch that bp_batch_workspace_bytes rejects."""
    from paper_1709_06509_amd import bpstereo as B

    L = B.library()
    B._batch_sigs(L)
    descs = (B.PairDesc * 3)()
    for i, (W, H, D) in enumerate([(64, 48, 16), (33, 21, 64), (26, 18, 128)]):
        descs[i] = B.PairDesc(0, 0, 0, 0, W, H, D, 0)
    for lam, trunc, bits in [(64, 4, 12), (4095, 1, 12), (1, 4095, 12), (4096, 1, 16), (1500, 4, 16), (5000, 4, 16)]:
        p = B.make_batch_params(5, 3, [6, 5, 4], lam, trunc)
        assert L.bp_batch_message_bits(descs, 3, ctypes.byref(p)) == bits, (lam, trunc)
    p = B.make_batch_params(5, 3, [6, 5, 4], 64, 4)
    assert L.bp_batch_message_bits(descs, 0, ctypes.byref(p)) == 0
    assert L.bp_batch_message_bits(descs, 3, ctypes.byref(B.make_batch_params(4, 3, [6, 5, 4], 64, 4))) == 0
