"""Helpers shared by the GPU tests: moving inputs to the device and comparing
GPU results with the oracle's."""
import sys

import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def bitmap_tensor(bm: np.ndarray) -> torch.Tensor:
    return dev(np.ascontiguousarray(bm, np.uint64).view(np.int64))


def say(*args) -> None:
    print(*args, flush=True)
    sys.stdout.flush()


def assert_bitmaps_equal(gpu: np.ndarray, ref: np.ndarray, what: str) -> None:
    gpu = np.asarray(gpu, np.uint64)
    ref = np.asarray(ref, np.uint64)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    diff = np.nonzero(gpu != ref)[0]
    assert len(diff) == 0, f"{what}: {len(diff)} words differ, first at {diff[:5]}"
