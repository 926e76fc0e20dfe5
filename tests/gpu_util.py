"""Shared helpers for the GPU tests (kept out of test collection)."""
import os
import sys

import numpy as np
import pytest


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def ctx():
    from paper_0905_2200_amd import fe
    return fe.Context(0)


def banner(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def oracle_counts(ids, ticks, num_types, cand, mode, projection=True):
    import oracle
    return oracle.count(ids, ticks, num_types, cand["types"], cand["len"], cand["lo"], cand["hi"],
                        mode, projection=projection)
