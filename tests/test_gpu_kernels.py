"""GPU parity of the building blocks through the C ABI: FFT vs the DFT
definition (numpy.fft), q = K p vs the oracle's assembled stiffness, z = M^+ r
vs a direct solve of the assembled M (lambda = 0, mu = 1/2), and the
projection G vs the small-strain appendix operator and dense brute force.
Shapes span several tiles with ragged tails (3D stencil tiles of 8 x 32 voxels
updating 7 x 31 nodes, 2D rows of 256 voxels updating 255 nodes, marches of
32-plane chunks along axis 0: operator shapes with n0 > 32 cross chunk
boundaries) and odd sizes (Nyquist-free axes, general radices)."""
import numpy as np
import pytest

from gpu_util import random_material, rel, say

pytestmark = pytest.mark.gpu

FFT_SHAPES = [(8, 8), (6, 10), (5, 7), (32, 32), (12, 9), (64, 512), (20, 13),
              (4, 6, 8), (3, 5, 7), (16, 16, 16), (8, 12, 10), (6, 20, 9), (2, 2, 2),
              # prime factors above 13 (direct-DFT passes)
              (17, 34), (151, 12), (34, 151), (4, 2039), (1661, 6), (17, 6, 34), (5, 151, 4),
              # the longest axes the LDS tiles take (first axis 2048 (FP64) / 3072 (FP32) in 2D,
              # last axis 4096)
              (2048, 16), (16, 4096), (1365, 3, 2)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_fft_roundtrip_matches_dft(shape, prec):
    import paper_2105_03297_amd as feh
    say("fft", shape, prec)
    if shape == (2048, 16) and prec == "fp32":
        shape = (3072, 16)
    dim = len(shape)
    L = 2
    h = feh.Homogenizer(shape, n_load=L, precision=prec)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((L * dim,) + shape)
    X = h.fft_forward(x.reshape(L * dim, -1)).cpu().numpy()
    ref = np.fft.rfftn(x, axes=tuple(range(1, dim + 1)))
    tol = 1e-13 if prec == "fp64" else 3e-6
    assert np.abs(X - ref).max() / np.abs(ref).max() < tol
    back = h.fft_inverse(ref.astype(np.complex128 if prec == "fp64" else np.complex64))
    np.testing.assert_allclose(back.cpu().numpy().reshape(x.shape), x, atol=tol * np.abs(x).max() * 10)
    h.close()


OP_SHAPES = [(6, 5), (7, 300), (40, 20), (3, 4, 5), (5, 9, 70), (18, 6, 5), (2, 2, 2), (9, 7, 130),
             (70, 9, 40), (65, 17, 33)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", OP_SHAPES)
def test_operator_matches_assembled_stiffness(shape, prec):
    import paper_2105_03297_amd as feh
    from oracle import fe
    say("operator", shape, prec)
    dim = len(shape)
    L = 2
    lam, mu = random_material(shape, 7, prec)
    hvox = (1.0, 1.3, 0.8)[:dim]
    h = feh.Homogenizer(shape, n_load=L, precision=prec, h=hvox)
    h.set_material(lam=lam, mu=mu)
    rng = np.random.default_rng(2)
    N = int(np.prod(shape))
    p = rng.standard_normal((L, N, dim))
    dt = np.float64 if prec == "fp64" else np.float32
    p = p.astype(dt).astype(np.float64)
    q = h.apply_operator(p).cpu().numpy().astype(np.float64)
    K = fe.assemble(lam, mu, hvox)
    Kabs = abs(K)
    for l in range(L):
        ref = (K @ p[l].ravel()).reshape(N, dim)
        if prec == "fp64":
            assert rel(q[l], ref) < 1e-13
        else:
            bound = (Kabs @ np.abs(p[l]).ravel()).reshape(N, dim)
            assert np.all(np.abs(q[l] - ref) <= 2e-6 * bound + 1e-30)
    h.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(5, 9, 70), (70, 9, 40), (65, 17, 33), (3, 40, 5)])
def test_operator_with_16_row_tiles_matches_assembled_stiffness(shape, prec):
    """The 3D stencil's taller tile (16 x 32 voxels, 512 threads, updating
    15 x 31 nodes; a tuning option) against the oracle's assembled stiffness,
    as the default tile above (ragged tiles, several x-chunks)."""
    import paper_2105_03297_amd as feh
    from oracle import fe
    say("operator, 16-row tiles", shape, prec)
    L = 2
    lam, mu = random_material(shape, 8, prec)
    hvox = (1.0, 1.3, 0.8)
    h = feh.Homogenizer(shape, n_load=L, precision=prec, h=hvox)
    t = feh.feh_plan_tuning(h.plan)
    t["stencil_rows"] = 16
    feh.feh_plan_set_tuning(h.plan, t)
    assert feh.feh_plan_tuning(h.plan)["stencil_rows"] == 16
    h.set_material(lam=lam, mu=mu)
    rng = np.random.default_rng(3)
    N = int(np.prod(shape))
    dt = np.float64 if prec == "fp64" else np.float32
    p = rng.standard_normal((L, N, 3)).astype(dt).astype(np.float64)
    q = h.apply_operator(p).cpu().numpy().astype(np.float64)
    h.close()
    K = fe.assemble(lam, mu, hvox)
    Kabs = abs(K)
    for l in range(L):
        ref = (K @ p[l].ravel()).reshape(N, 3)
        if prec == "fp64":
            assert rel(q[l], ref) < 1e-13
        else:
            bound = (Kabs @ np.abs(p[l]).ravel()).reshape(N, 3)
            assert np.all(np.abs(q[l] - ref) <= 2e-6 * bound + 1e-30)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_operator_on_the_largest_planes(prec):
    """q = K p on the largest planes a 3D plan takes (4096 x 4096 in FP32,
    4096 x 2048 in FP64, where the last-axis transform of 3 components
    reaches the LDS tile; 64 MiB per component plane, both axes ragged against
    the 7 x 31-node tiles), at 96 sampled nodes (the plane's last row and
    column, its far corner, tile borders and random nodes) against the
    oracle's element sums at those nodes."""
    import paper_2105_03297_amd as feh
    from oracle import fe
    say("operator, largest planes", prec)
    shape = (3, 4096, 4096) if prec == "fp32" else (3, 4096, 2048)
    dt = np.float64 if prec == "fp64" else np.float32
    rng = np.random.default_rng(11)
    E = rng.uniform(1.0, 10.0, shape)
    lam, mu = fe.lame(E, 0.3)
    lam = lam.astype(dt).astype(np.float64)
    mu = mu.astype(dt).astype(np.float64)
    h = feh.Homogenizer(shape, n_load=1, precision=prec)
    h.set_material(lam=lam, mu=mu)
    N = int(np.prod(shape))
    p = rng.standard_normal((N, 3)).astype(dt)
    q = h.apply_operator(p.reshape(1, N, 3)).cpu().numpy()[0].astype(np.float64)
    h.close()
    n1, n2 = shape[1], shape[2]
    picks = [(x, y, z) for x in range(3) for (y, z) in [(n1 - 1, n2 - 1), (0, 0), (n1 - 1, 0), (0, n2 - 1),
                                                       (7, 31), (6, 30), (n1 - 1, n2 - 4), (n1 - 2, n2 - 1)]]
    picks += [tuple(int(v) for v in c) for c in zip(rng.integers(0, 3, 72), rng.integers(0, n1, 72), rng.integers(0, n2, 72))]
    nodes = np.array([np.ravel_multi_index(c, shape) for c in picks])
    ref = fe.apply_K_at_nodes(lam, mu, p.astype(np.float64), nodes)
    err = np.abs(q[nodes] - ref).max() / np.abs(ref).max()
    print(prec, "largest planes: max error at %d nodes relative to max |K p| %.3e" % (len(nodes), err))
    assert err < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(8, 8), (6, 5), (16, 300), (4, 6, 8), (5, 3, 7), (20, 9, 70)])
def test_preconditioner_matches_direct_solve(shape, prec):
    """z = M^+ r with M the FE stiffness of lambda = 0, mu = 1/2 (B^T B)."""
    import paper_2105_03297_amd as feh
    from oracle import fe
    say("precond", shape, prec)
    dim = len(shape)
    L = 2
    hvox = (1.0, 0.7, 1.2)[:dim]
    h = feh.Homogenizer(shape, n_load=L, precision=prec, h=hvox)
    rng = np.random.default_rng(4)
    N = int(np.prod(shape))
    r = rng.standard_normal((L, N, dim))
    z = h.apply_preconditioner(r).cpu().numpy().astype(np.float64)
    M = fe.assemble(np.zeros(shape), np.full(shape, 0.5), hvox)
    tol = 1e-11 if prec == "fp64" else 2e-5
    for l in range(L):
        rr = r[l] - r[l].mean(axis=0)
        ref = fe.solve_direct(M, rr.ravel(), dim).reshape(N, dim)
        assert rel(z[l], ref) < tol
        assert np.abs(z[l].mean(axis=0)).max() < tol * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(4, 4), (5, 4), (9, 7), (3, 4, 5), (4, 4, 4), (6, 5, 8)])
def test_projection_matches_appendix_operator(shape, prec):
    """G on element strain fields: GPU (factored, real-space B and B^T, FFT
    only for (B^T B)^+) vs the small-strain appendix formula G_{TL,ijlm}
    applied per wavevector; idempotence on the GPU."""
    import paper_2105_03297_amd as feh
    from oracle import projection as pj
    say("projection", shape, prec)
    dim = len(shape)
    ne = 2 if dim == 2 else 6
    L = 1
    h = feh.Homogenizer(shape, n_load=L, precision=prec)
    rng = np.random.default_rng(6)
    e = rng.standard_normal(shape + (ne, dim, dim))
    e = 0.5 * (e + np.swapaxes(e, -1, -2))
    N = int(np.prod(shape))
    Ge = h.apply_projection(e.reshape(1, N, ne, dim, dim)).cpu().numpy().astype(np.float64)
    G = pj.small_strain_operator(pj.symbols("fe", shape))
    ref = pj.apply_small_strain(G, e).reshape(N, ne, dim, dim)
    tol = 1e-12 if prec == "fp64" else 3e-5
    assert rel(Ge[0], ref) < tol
    GGe = h.apply_projection(Ge).cpu().numpy().astype(np.float64)
    assert rel(GGe[0], Ge[0]) < tol
    if N * dim <= 200:
        Gd = pj.dense_projection(shape)
        assert rel(Ge[0].ravel(), Gd @ e.ravel()) < tol
    h.close()


def test_stream_copy_is_exact_and_checks_arguments():
    """The measurement copy moves every byte; misaligned, ragged or
    overlapping requests are rejected."""
    import torch
    import paper_2105_03297_amd as feh
    say("stream copy")
    st = torch.cuda.current_stream().cuda_stream
    for n in (16, 4096 + 16, (1 << 22) + 48):
        src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros(n + 32, dtype=torch.uint8, device="cuda")
        feh.feh_stream_copy(dst.data_ptr(), src.data_ptr(), n, st)
        torch.cuda.synchronize()
        assert torch.equal(dst[:n], src) and int(dst[n:].sum()) == 0
    buf = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    for d, s_, n in ((buf.data_ptr() + 512, buf.data_ptr(), 24), (buf.data_ptr() + 520, buf.data_ptr(), 16),
                     (buf.data_ptr() + 256, buf.data_ptr(), 512), (0, buf.data_ptr(), 16)):
        with pytest.raises(feh.FehError) as ei:
            feh.feh_stream_copy(d, s_, n, st)
        assert ei.value.status == feh.FEH_EINVAL
