"""Helpers shared by the GPU tests: a context fixture and parity checks."""
import sys

import numpy as np
import torch

import oracle
import paper_2310_13870_amd as fsg

BAND = 1e-6  # a sample whose oracle path passes within 1e-6 of a split boundary is band-exempt


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def compare_neighbours(nbr_gpu, nbr_ref, margin_ref):
    """Returns (mismatch, band_exempt_mismatch, non_exempt_mismatch)."""
    nbr_gpu = np.asarray(nbr_gpu)
    nbr_ref = np.asarray(nbr_ref)
    mism = nbr_gpu != nbr_ref
    exempt = np.asarray(margin_ref) < BAND
    return int(mism.sum()), int((mism & exempt).sum()), int((mism & ~exempt).sum())
