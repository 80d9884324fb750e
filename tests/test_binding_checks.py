"""Host-side checks of the Python binding: caller-supplied output tensors are
validated against the stack (T frames, W = 2w-1 shifts per axis, the frames'
device) before any pointer reaches the C ABI, since the kernels write exactly
T rows of each output and would write past a smaller one.  Runs on the CPU
(the checks are pure host logic; CPU tensors stand in for device tensors)."""
import pytest
import torch

from paper_1506_06039_amd import moco

CPU = torch.device("cpu")


def _good(T=5, W=7, surface=True):
    return moco.Result(
        shifts=torch.zeros((T, 2), dtype=torch.int32), fmin=torch.zeros(T, dtype=torch.float64),
        frefine=torch.zeros((T, 9), dtype=torch.float64),
        coarse=torch.zeros((T, 2), dtype=torch.int32),
        gaps=torch.zeros((T, 2), dtype=torch.float64),
        fsurf=torch.zeros((T, W, W), dtype=torch.float64) if surface else None,
        recomputed=torch.zeros(T, dtype=torch.int32))


def test_valid_result_passes():
    moco._validate_result(_good(), 5, 7, CPU)
    moco._validate_result(_good(surface=False), 5, 7, CPU)
    r = _good()
    r.recomputed = None
    moco._validate_result(r, 5, 7, CPU)


@pytest.mark.parametrize("field,bad", [
    ("shifts", torch.zeros((4, 2), dtype=torch.int32)),          # a smaller stack's result
    ("shifts", torch.zeros((5, 2), dtype=torch.int64)),          # wrong dtype
    ("fmin", torch.zeros(5, dtype=torch.float32)),               # float32 fmin
    ("frefine", torch.zeros((5, 9), dtype=torch.float64)[:, :8]),  # wrong shape
    ("frefine", torch.zeros((9, 5), dtype=torch.float64).t()),   # non-contiguous view
    ("gaps", torch.zeros((5, 1), dtype=torch.float64)),
    ("coarse", torch.zeros((5, 2), dtype=torch.float32)),
    ("fsurf", torch.zeros((5, 5, 5), dtype=torch.float64)),      # surface of another window
    ("recomputed", torch.zeros(6, dtype=torch.int32)),
])
def test_bad_output_rejected(field, bad):
    r = _good()
    setattr(r, field, bad)
    with pytest.raises(ValueError):
        moco._validate_result(r, 5, 7, CPU)


def test_missing_required_output_rejected():
    r = _good()
    r.gaps = None
    with pytest.raises(ValueError):
        moco._validate_result(r, 5, 7, CPU)


def test_wrong_device_rejected():
    with pytest.raises(ValueError):
        moco._validate_result(_good(), 5, 7, torch.device("cuda", 0))


def test_apply_outputs_checked_before_the_call():
    # frames on the CPU are refused first; the output checks use the same helper
    fr = torch.zeros((2, 4, 4), dtype=torch.uint16)
    with pytest.raises(ValueError):
        moco._check_tensor("out", torch.zeros((2, 4, 5), dtype=torch.uint16), (2, 4, 4),
                           fr.dtype, CPU)
    with pytest.raises(ValueError):
        moco._check_tensor("mean_out", torch.zeros((4, 4), dtype=torch.float32), (4, 4),
                           torch.float64, CPU)
    moco._check_tensor("out", torch.zeros((2, 4, 4), dtype=torch.uint16), (2, 4, 4),
                       fr.dtype, CPU)
