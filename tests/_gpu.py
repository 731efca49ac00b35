"""Helpers for the GPU parity tests: host<->device moves and the relative-error check.

Parity bar (FP64): max |gpu - oracle| <= tol * max |oracle| per field, tol = 1e-12 unless a
test states otherwise; integer decisions are compared bit for bit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(g, r):
    g = np.asarray(g); r = np.asarray(r)
    scale = np.abs(r).max()
    return np.abs(g - r).max() / (scale if scale > 0 else 1.0)


def assert_parity(g, r, tol=1e-12, what=""):
    e = rel_err(g, r)
    assert e <= tol, "%s: relative error %.3e > %.1e" % (what, e, tol)
    return e


def announce(msg):
    print(msg, flush=True)
    sys.stdout.flush()
