"""Helpers shared by the GPU parity tests (no method arithmetic)."""
import os

import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1710_03757_amd as m
    return torch, m


def log(msg):
    print(msg, flush=True)
