"""The allocation-free exact matvec (h2ulv_matvec_exact_noalloc) against the
allocating one (h2ulv_matvec_exact), called through the C-ABI: two calls in a
row on one GPU, the second with a smaller input, both large enough that the
split partial sums go through the per-GPU array; a third with one column at
n = 2^20 (the single-column pair form's slots); then a request beyond the
array's size, rejected before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from paper_2208_10907_amd import h2ulv as H

pytestmark = pytest.mark.gpu


def _factor(n, seed):
    X = W.cube_points(n, seed)
    # a cheap factorization: only its points and kernel are used here
    return H.factorize(X, H.make_params(leaf=256, tol=1e-2, rank_cap=16, far_sample=8))


def _like(x, fill):
    y = torch.full((x.shape[1], x.shape[0]), fill, dtype=x.dtype, device=x.device)
    return y.t()  # column-major like x


def _ld(t):
    # leading dimension of a column-major block; a single column's stride along
    # the column index is not meaningful (torch may report 1), so it is n
    return t.stride(1) if t.shape[1] > 1 else t.shape[0]


def _reference(f, x):
    y = _like(x, 0.0)
    st = H.lib().h2ulv_matvec_exact(f._h, C.c_void_p(x.data_ptr()), _ld(x),
                                    C.c_void_p(y.data_ptr()), _ld(y), x.shape[1], None)
    assert st == H.OK, H.lib().h2ulv_last_error()
    return y


def _noalloc(f, x):
    y = _like(x, float("nan"))
    st = H.lib().h2ulv_matvec_exact_noalloc(f._h, C.c_void_p(x.data_ptr()), _ld(x),
                                            C.c_void_p(y.data_ptr()), _ld(y), x.shape[1],
                                            None)
    assert st == H.OK, H.lib().h2ulv_last_error()
    torch.cuda.synchronize()
    return y


def _cols(n, nrhs, seed):
    x = torch.tensor(W.gaussian_rhs(n, nrhs, seed), device="cuda")
    return x.t().contiguous().t()  # column-major (Fortran order), stride (1, n)


def test_noalloc_matvec_equals_allocating_matvec():
    # first call: n = 131072, 8 columns, 8 splits (half the array)
    fa = _factor(131072, 21)
    xa = _cols(131072, 8, 22)
    ya = _noalloc(fa, xa)
    ra = _reference(fa, xa)
    torch.cuda.synchronize()
    assert torch.isfinite(ya).all()
    assert torch.equal(ya, ra)
    # second call, smaller input (n = 65536, 3 columns): the array keeps the first
    # call's partial sums, which must not leak into this result
    fb = _factor(65536, 23)
    xb = _cols(65536, 3, 24)
    yb = _noalloc(fb, xb)
    rb = _reference(fb, xb)
    torch.cuda.synchronize()
    assert torch.equal(yb, rb)
    # and against the definition of the matrix on sampled rows
    from oracle import h2ulv_ref as O
    Xb = W.cube_points(65536, 23)
    rows = np.random.default_rng(5).choice(65536, 24, replace=False)
    yo = O.kernel_block(Xb, rows, np.arange(65536), O.Params()) @ xb.cpu().numpy()
    assert np.linalg.norm(yb.cpu().numpy()[rows] - yo) / np.linalg.norm(yo) < 1e-14
    # third call: one column at n = 2^20, the single-column pair form, whose y_I
    # and y_J slots (9 n doubles, over half the array) go through it
    fd = _factor(1 << 20, 27)
    xd = _cols(1 << 20, 1, 28)
    yd = _noalloc(fd, xd)
    rd = _reference(fd, xd)
    torch.cuda.synchronize()
    assert torch.equal(yd, rd)
    del fd
    # a request whose partial sums exceed the array is refused before any launch
    # (n = 262144, 8 columns: the 8-column pair form's 72 n doubles)
    fc = _factor(262144, 25)
    xc = _cols(262144, 8, 26)
    yc = _like(xc, 0.0)
    st = H.lib().h2ulv_matvec_exact_noalloc(fc._h, C.c_void_p(xc.data_ptr()), xc.stride(1),
                                            C.c_void_p(yc.data_ptr()), yc.stride(1), 8, None)
    assert st == H.ERR_INVALID_ARG
    assert b"allocation-free" in H.lib().h2ulv_last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(yc) == 0
