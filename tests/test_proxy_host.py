"""Host logic of the proxy's library entry points, without a GPU: the
training step's workspace plan and the argument checks that refuse a call
before anything is launched."""
import ctypes

import pytest

from paper_2510_12897_amd import opf

OPF_E_ARG = opf.OPF_E_ARG


def _desc(dims, flat=4096, flat_bf16=8192):
    arr = (ctypes.c_int32 * len(dims))(*dims)
    d = opf.MlpDesc(len(dims) - 1, arr, flat, flat_bf16, 16384, 32768, 65536)
    return d, arr


def _bytes(dims, B, **kw):
    d, keep = _desc(dims, **kw)
    out = ctypes.c_int64(-1)
    rc = opf.lib().prox_train_step_bytes(ctypes.byref(d), B, ctypes.byref(out))
    return rc, out.value


def test_train_step_workspace_grows_with_the_batch():
    dims = [600, 1024, 1024, 1024, 720]
    rc1, b1 = _bytes(dims, 4096)
    rc2, b2 = _bytes(dims, 8192)
    assert rc1 == rc2 == 0
    # at least the FP32 pre-activations, the FP32 loss gradient and the
    # parameter gradient of a 4,096-sample step
    n_params = sum(fo * fi + fo for fi, fo in zip(dims[:-1], dims[1:]))
    assert b1 >= 4 * 4096 * sum(dims[1:]) + 4 * 4096 * 720 + 4 * n_params
    assert b2 > b1 and b1 % 256 == 0


@pytest.mark.parametrize("dims,B,msg", [
    ([600, 1024, 720], 4094, "multiple of 4"),
    ([600, 1024, 720], 0, "multiple of 4"),
    ([602, 1024, 720], 4096, "multiples of 4"),
])
def test_train_step_plan_refusals(dims, B, msg):
    rc, _ = _bytes(dims, B)
    assert rc == OPF_E_ARG
    assert msg in opf.lib().opf_last_error().decode()


def test_train_step_refuses_misaligned_bf16_weights():
    # widths 28 -> 68 -> 64 -> 40: layer 2 reads BF16 weights (input width
    # 64) at parameter offset 68*28 + 68 + 64*68 + 64 = 6388, not a multiple
    # of 8 elements, so its 16-byte loads would straddle
    rc, _ = _bytes([28, 68, 64, 40], 64)
    assert rc == OPF_E_ARG
    assert "16-byte aligned" in opf.lib().opf_last_error().decode()
    # without a BF16 copy the same widths plan
    rc, b = _bytes([28, 68, 64, 40], 64, flat_bf16=None)
    assert rc == 0 and b > 0


def test_gemm_gelu_bwd_argument_checks():
    L = opf.lib()
    p = 4096  # a 16-byte aligned stand-in address: the checks refuse before any launch
    assert L.prox_gemm_gelu_bwd(p, 1, 12, p, 0, 64, p, 64, p, 64, 128, 64, 12, p, None) == OPF_E_ARG
    assert "multiples of 8" in L.opf_last_error().decode()
    assert L.prox_gemm_gelu_bwd(p, 0, 64, p, 0, 62, p, 64, p, 64, 128, 64, 64, p, None) == OPF_E_ARG
    assert L.prox_gemm_gelu_bwd(None, 0, 64, p, 0, 64, p, 64, p, 64, 128, 64, 64, p, None) == OPF_E_ARG
    assert L.prox_gemm_gelu_bwd(p + 4, 0, 64, p, 0, 64, p, 64, p, 64, 128, 64, 64, p, None) == OPF_E_ARG
    assert L.prox_colsum_parts(p, 0, 64, p, 1.0, None) == OPF_E_ARG


def test_sampling_and_scaling_argument_checks():
    L = opf.lib()
    p = 4096
    assert L.prox_sample_loads(p, p, p, 0.3, 0, 300, p, p, None) == OPF_E_ARG
    assert L.prox_sample_loads(None, p, p, 0.3, 8, 300, p, p, None) == OPF_E_ARG
    assert L.prox_scale_rows(p, None, 8, 16, p, None) == OPF_E_ARG
