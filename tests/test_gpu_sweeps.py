"""The fused four-sweep smoother of the multigrid solve (Sec. 2.1 Eq. 4),
one z-marching pass with its planes in LDS, against four single-colour
launches on the same inputs (bit-identical over the whole array) and against
red-black Gauss-Seidel written out here in FP64 from its definition, for the
zero initial guess and a given one, and in its pre-smoothing form with the
red residual of the result (against the separate residual kernel, and the
residual of the FP64 sweeps), at 64^3 .. 256^3 (chunks of 16 planes,
several columns along every axis, periodic wrap at every face)."""
import numpy as np
import pytest

from helpers import log

pytestmark = pytest.mark.gpu


def _split(a):
    """(k, j, i) array -> colour-split vector: red cells ((i+j+k) even) in
    row order, then black ones (half index i >> 1 within a row)."""
    k, j, i = np.indices(a.shape)
    red = ((i + j + k) & 1) == 0
    return np.concatenate([a[red], a[~red]])


def _unsplit(v, n):
    k, j, i = np.indices((n, n, n))
    red = ((i + j + k) & 1) == 0
    a = np.empty((n, n, n), v.dtype)
    a[red] = v[: n**3 // 2]
    a[~red] = v[n**3 // 2:]
    return a


def _rbgs(e, r, scale, inv_diag, first):
    """Red, black, red, black: each cell of the colour set to
    (sum of its 6 periodic neighbours - scale r) * inv_diag."""
    e = np.zeros_like(r) if first else e.copy()
    k, j, i = np.indices(r.shape)
    red = ((i + j + k) & 1) == 0
    for colour in (red, ~red, red, ~red):
        nb = sum(np.roll(e, s, axis=a) for a in range(3) for s in (1, -1))
        e[colour] = ((nb - scale * r) * inv_diag)[colour]
    return e


@pytest.mark.parametrize("n", [64, 128, 256])
@pytest.mark.parametrize("first", [True, False])
def test_fused_sweeps_match_single_colour_sweeps(n, first):
    import torch
    import paper_1709_04703_amd as P

    rng = np.random.Generator(np.random.PCG64(4703 + n))
    e0 = rng.uniform(-1.0, 1.0, n**3).astype(np.float32)
    r = rng.uniform(-1.0, 1.0, n**3).astype(np.float32)
    scale = 4.0                                   # level 1 of a hierarchy
    inv_diag = float(np.float32(1.0 / (6.0 + scale * 0.113)))
    e_t = torch.as_tensor(e0).cuda()
    r_t = torch.as_tensor(r).cuda()
    fused = torch.full_like(e_t, float("nan"))
    single = e_t.clone()
    P.rb_sweeps(n, e_t, fused, r_t, scale, inv_diag, first, True)
    P.rb_sweeps(n, e_t, single, r_t, scale, inv_diag, first, False)
    torch.cuda.synchronize()
    a = fused.cpu().numpy()
    b = single.cpu().numpy()
    assert np.array_equal(e_t.cpu().numpy().view(np.uint32), e0.view(np.uint32))   # input kept
    nd = int(np.count_nonzero(a.view(np.uint32) != b.view(np.uint32)))
    log(f"rb_sweeps n={n} first={first}: {nd} of {n**3} differ between fused and single-colour")
    assert nd == 0
    if n <= 128:
        ref = _rbgs(_unsplit(e0, n).astype(np.float64), _unsplit(r, n).astype(np.float64), scale,
                    inv_diag, first)
        err = np.abs(_unsplit(a, n).astype(np.float64) - ref).max() / np.abs(ref).max()
        log(f"rb_sweeps n={n} first={first}: max error vs FP64 definition {err:.2e}")
        assert err < 1e-5


@pytest.mark.parametrize("n", [64, 128, 256])
@pytest.mark.parametrize("first", [True, False])
def test_fused_sweeps_with_residual(n, first):
    # the pre-smoothing form: the red residual of the result goes to t (red
    # half) and the fused pass leaves e's red half unwritten
    import torch
    import paper_1709_04703_amd as P

    rng = np.random.Generator(np.random.PCG64(9000 + n))
    e0 = rng.uniform(-1.0, 1.0, n**3).astype(np.float32)
    r = rng.uniform(-1.0, 1.0, n**3).astype(np.float32)
    scale, kappa_h2 = 4.0, 0.113
    inv_diag = float(np.float32(1.0 / (6.0 + scale * kappa_h2)))
    e_t = torch.as_tensor(e0).cuda()
    r_t = torch.as_tensor(r).cuda()
    fused, t_f = torch.full_like(e_t, float("nan")), torch.full_like(e_t, float("nan"))
    single, t_s = e_t.clone(), torch.full_like(e_t, float("nan"))
    P.rb_sweeps(n, e_t, fused, r_t, scale, inv_diag, first, True, t_f, kappa_h2)
    P.rb_sweeps(n, e_t, single, r_t, scale, inv_diag, first, False, t_s, kappa_h2)
    torch.cuda.synchronize()
    h = n**3 // 2
    a, b = fused.cpu().numpy(), single.cpu().numpy()
    ta, tb = t_f.cpu().numpy(), t_s.cpu().numpy()
    nd_e = int(np.count_nonzero(a[h:].view(np.uint32) != b[h:].view(np.uint32)))
    nd_t = int(np.count_nonzero(ta[:h].view(np.uint32) != tb[:h].view(np.uint32)))
    log(f"rb_sweeps + residual n={n} first={first}: black e {nd_e}, red t {nd_t} of {h} differ")
    assert nd_e == 0 and nd_t == 0
    assert np.isnan(ta[h:]).all()                    # black half of t not written
    if n <= 128:
        ref = _rbgs(_unsplit(e0, n).astype(np.float64), _unsplit(r, n).astype(np.float64), scale,
                    inv_diag, first)
        k, j, i = np.indices(ref.shape)
        red = ((i + j + k) & 1) == 0
        nb = sum(np.roll(ref, sh, axis=ax) for ax in range(3) for sh in (1, -1))
        tref = _unsplit(r, n).astype(np.float64) - (nb - 6.0 * ref) / scale + kappa_h2 * ref
        got = _unsplit(np.concatenate([ta[:h], np.zeros(h, np.float32)]), n).astype(np.float64)
        err = np.abs(got[red] - tref[red]).max() / np.abs(tref[red]).max()
        log(f"rb_sweeps + residual n={n} first={first}: max t error vs FP64 {err:.2e}")
        assert err < 1e-5


def _rbgs_box(e, r, scale, inv_diag, first, lo, hi):
    """_rbgs with e = 0 outside the box lo..hi (inclusive, (x, y, z)) and
    only its cells swept."""
    k, j, i = np.indices(r.shape)
    inside = ((i >= lo[0]) & (i <= hi[0]) & (j >= lo[1]) & (j <= hi[1]) & (k >= lo[2]) & (k <= hi[2]))
    e = np.where(inside, 0.0 if first else e, 0.0)
    red = ((i + j + k) & 1) == 0
    for colour in (red, ~red, red, ~red):
        nb = sum(np.roll(e, s_, axis=a) for a in range(3) for s_ in (1, -1))
        upd = colour & inside
        e[upd] = ((nb - scale * r) * inv_diag)[upd]
    return e, inside


@pytest.mark.parametrize("n,lo,hi", [(128, (5, 9, 3), (118, 101, 124)),
                                     (256, (17, 1, 30), (230, 254, 201))])
@pytest.mark.parametrize("first,resid", [(True, True), (False, True), (False, False)])
def test_fused_sweeps_on_a_frozen_exterior_box(n, lo, hi, first, resid):
    # the shrinking domain's levels: e is zero outside the box and stays so
    import torch
    import paper_1709_04703_amd as P

    rng = np.random.Generator(np.random.PCG64(7000 + n + 2 * first + resid))
    k, j, i = np.indices((n, n, n))
    inside = ((i >= lo[0]) & (i <= hi[0]) & (j >= lo[1]) & (j <= hi[1]) & (k >= lo[2]) & (k <= hi[2]))
    e_full = np.where(inside, rng.uniform(-1.0, 1.0, (n, n, n)), 0.0).astype(np.float32)
    e0 = _split(e_full)
    r = rng.uniform(-1.0, 1.0, n**3).astype(np.float32)
    scale, kappa_h2 = 1.0, 0.113
    inv_diag = float(np.float32(1.0 / (6.0 + scale * kappa_h2)))
    e_t, r_t = torch.as_tensor(e0).cuda(), torch.as_tensor(r).cuda()
    fused, single = torch.zeros_like(e_t), e_t.clone()
    t_f = torch.zeros_like(e_t) if resid else None
    t_s = torch.zeros_like(e_t) if resid else None
    P.rb_sweeps(n, e_t, fused, r_t, scale, inv_diag, first, True, t_f, kappa_h2, box=(lo, hi))
    P.rb_sweeps(n, e_t, single, r_t, scale, inv_diag, first, False, t_s, kappa_h2, box=(lo, hi))
    torch.cuda.synchronize()
    h = n**3 // 2
    a, b = fused.cpu().numpy(), single.cpu().numpy()
    part = slice(h, None) if resid else slice(None)        # with the residual: black e only
    nd = int(np.count_nonzero(a[part].view(np.uint32) != b[part].view(np.uint32)))
    msg = f"rb_sweeps box n={n} first={first} resid={resid}: e {nd}"
    if resid:
        ta, tb = t_f.cpu().numpy(), t_s.cpu().numpy()
        ndt = int(np.count_nonzero(ta[:h].view(np.uint32) != tb[:h].view(np.uint32)))
        msg += f", t {ndt}"
        nd += ndt
    log(msg + " entries differ")
    assert nd == 0
    out = _unsplit(a, n)
    if not resid:
        assert np.all(out[~inside] == 0.0)               # the exterior stays zero
    if n <= 128:
        ref, ins = _rbgs_box(_unsplit(e0, n).astype(np.float64), _unsplit(r, n).astype(np.float64),
                             scale, inv_diag, first, lo, hi)
        sel = ins if not resid else ins & (((i + j + k) & 1) == 1)
        err = np.abs(out[sel].astype(np.float64) - ref[sel]).max() / np.abs(ref[sel]).max()
        log(f"rb_sweeps box n={n}: max error vs FP64 {err:.2e}")
        assert err < 1e-5


def test_fused_sweeps_in_place_first():
    # from the zero guess the fused pass may write the array it was given
    import torch
    import paper_1709_04703_amd as P

    n = 128
    rng = np.random.Generator(np.random.PCG64(7))
    r = torch.as_tensor(rng.uniform(-1.0, 1.0, n**3).astype(np.float32)).cuda()
    e = torch.full((n**3,), float("nan"), device="cuda")
    ref = torch.full_like(e, float("nan"))
    P.rb_sweeps(n, e, e, r, 1.0, 1.0 / 6.0, True, True)
    P.rb_sweeps(n, None, ref, r, 1.0, 1.0 / 6.0, True, False)
    torch.cuda.synchronize()
    assert torch.equal(e.view(torch.int32), ref.view(torch.int32))
