"""Differentiable GW iteration: torch.autograd.Functions over the libqgw calls.

Each Function's forward calls a libqgw step and its backward calls the
matching ``*_bwd`` entry point; PyTorch only chains them and holds the
tensors.  Cotangents follow PyTorch's complex convention
(zbar = dL/dRe z + i dL/dIm z), which is the library's.  FP64 plans only.

The iteration (Fig. fig-self (b)) is composed from the steps exactly as the
library's composite call runs it:

    n(k) = Herm(-G(beta^-)), n(R), Sigma_HF(R) -> Sigma_HF(k)
    G(tau), G(beta - tau) -> R, P(q, tau), P(q, i nu), W^C(q, i nu), W^C(q, tau)
    Sigma^C(k, tau) -> Sigma^C(k, i w) (Hermitian part), then G and mu from
    the Dyson equation at the target filling.

``run`` unrolls n iterations from G0 with per-iteration checkpointing: only
G(i w) of each iteration is stored, the intermediates are recomputed in the
backward pass.  The chemical potential enters through the implicit function
N_e(mu, H, Sigma) = N_target (the Dyson-G adjoint carries that term).
"""
import torch
from torch.utils.checkpoint import checkpoint

from . import qgw


def _new(shape, like):
    return torch.empty(shape, dtype=like.dtype, device=like.device)


def _c(x):
    return x if x.is_contiguous() else x.contiguous()


class DLR(torch.autograd.Function):
    """out = scale T_map x over the node axis (a1, a11, density row)."""

    @staticmethod
    def forward(ctx, plan, which, x, scale, hermitian):
        rows = 1 if which == qgw.F_IW2BETA else plan.r
        out = _new((rows,) + tuple(x.shape[1:]), x)
        plan.dlr_transform(which, _c(x), out, scale, hermitian)
        ctx.args = (plan, which, scale, hermitian, tuple(x.shape))
        return out

    @staticmethod
    def backward(ctx, gy):
        plan, which, scale, hermitian, shape = ctx.args
        gx = torch.empty(shape, dtype=gy.dtype, device=gy.device)
        plan.dlr_transform_bwd(which, _c(gy), gx, scale, hermitian)
        return None, None, gx, None, None


class DLRPairs(torch.autograd.Function):
    """a5 / a7 on pair arrays, with the slab <-> matrix layout change."""

    @staticmethod
    def forward(ctx, plan, which, in_layout, out_layout, x):
        out = _new(_pair_shape(plan, out_layout), x)
        plan.dlr_transform_pairs(which, in_layout, out_layout, _c(x), out)
        ctx.args = (plan, which, in_layout, out_layout)
        return out

    @staticmethod
    def backward(ctx, gy):
        plan, which, in_layout, out_layout = ctx.args
        gx = _new(_pair_shape(plan, in_layout), gy)
        plan.dlr_transform_pairs_bwd(which, in_layout, out_layout, _c(gy), gx)
        return None, None, None, None, gx


def _pair_shape(plan, layout, nodes=None):
    r = plan.r if nodes is None else nodes
    if layout == qgw.LAYOUT_SLAB:
        return (r, plan.n_b, plan.n_b, plan.n_k)
    return (r, plan.n_k, plan.n_b, plan.n_b)


class FFT(torch.autograd.Function):
    """Lattice transform over the trailing N_k axis (Eq. eq:fourier-transform-kr)."""

    @staticmethod
    def forward(ctx, plan, direction, x):
        out = torch.empty_like(x)
        plan.lattice_fft(direction, _c(x), out)
        ctx.args = (plan, direction)
        return out

    @staticmethod
    def backward(ctx, gy):
        plan, direction = ctx.args
        gx = torch.empty_like(gy)
        plan.lattice_fft_bwd(direction, _c(gy), gx)
        return None, None, gx


class PairLayout(torch.autograd.Function):
    """Static pair array [N_b][N_b][N_k] -> [N_k][N_b][N_b] (a permutation)."""

    @staticmethod
    def forward(ctx, plan, x):
        out = _new((plan.n_k, plan.n_b, plan.n_b), x)
        plan.pair_layout(_c(x), out, qgw.LAYOUT_SLAB, qgw.LAYOUT_MATRIX)
        ctx.plan = plan
        return out

    @staticmethod
    def backward(ctx, gy):
        plan = ctx.plan
        gx = _new((plan.n_b, plan.n_b, plan.n_k), gy)
        plan.pair_layout(_c(gy), gx, qgw.LAYOUT_MATRIX, qgw.LAYOUT_SLAB)
        return None, gx


class Bubble(torch.autograd.Function):
    """a3 + a4: P(q, tau) from G(R, tau) and G(R, beta - tau)."""

    @staticmethod
    def forward(ctx, plan, gt, gr):
        gt, gr = _c(gt), _c(gr)
        out = _new(_pair_shape(plan, qgw.LAYOUT_SLAB), gt)
        plan.bubble(gt, gr, out, out_q=True)
        ctx.save_for_backward(gt, gr)
        ctx.plan = plan
        return out

    @staticmethod
    def backward(ctx, gp):
        gt, gr = ctx.saved_tensors
        a, b = torch.empty_like(gt), torch.empty_like(gr)
        ctx.plan.bubble_bwd(gt, gr, _c(gp), a, b)
        return None, a, b


class Sigma(torch.autograd.Function):
    """a8-a10: Sigma^C(k, tau) from G(R, tau) and W^C(q, tau)."""

    @staticmethod
    def forward(ctx, plan, gt, wc):
        gt, wc = _c(gt), _c(wc)
        out = torch.empty_like(gt)
        plan.sigma(gt, wc, out, in_q=True, out_k=True)
        ctx.save_for_backward(gt, wc)
        ctx.plan = plan
        return out

    @staticmethod
    def backward(ctx, gs):
        gt, wc = ctx.saved_tensors
        a, b = torch.empty_like(gt), torch.empty_like(wc)
        ctx.plan.sigma_bwd(gt, wc, _c(gs), a, b, out_k=True)
        return None, a, b


class DysonW(torch.autograd.Function):
    """a6: W^C(q, i nu) from V(q) (matrix layout) and P(q, i nu)."""

    @staticmethod
    def forward(ctx, plan, vq, pnu):
        vq, pnu = _c(vq), _c(pnu)
        out = torch.empty_like(pnu)
        plan.dyson_W(vq, pnu, out)
        ctx.save_for_backward(vq, pnu)
        ctx.plan = plan
        return out

    @staticmethod
    def backward(ctx, gw):
        vq, pnu = ctx.saved_tensors
        a, b = torch.empty_like(pnu), torch.empty_like(vq)
        ctx.plan.dyson_W_bwd(vq, pnu, _c(gw), a, b)
        return None, b, a


class HartreeFock(torch.autograd.Function):
    """a12: Sigma_HF(R) from V(R) and n(R)."""

    @staticmethod
    def forward(ctx, plan, v_r, n_r):
        v_r, n_r = _c(v_r), _c(n_r)
        out = torch.empty_like(n_r)
        plan.hartree_fock(v_r, n_r, out)
        ctx.save_for_backward(v_r, n_r)
        ctx.plan = plan
        return out

    @staticmethod
    def backward(ctx, gs):
        v_r, n_r = ctx.saved_tensors
        nb, vb = torch.empty_like(n_r), torch.empty_like(v_r)
        ctx.plan.hartree_fock_bwd(v_r, n_r, _c(gs), nb, vb)
        return None, vb, nb


class Add(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, a, b):
        out = torch.empty_like(a)
        plan.add(_c(a), _c(b), out)
        return out

    @staticmethod
    def backward(ctx, g):
        return None, g, g


class DysonG(torch.autograd.Function):
    """a13: G(k, i w) and mu at the target filling from H(k) and Sigma^C(k, i w).

    Returns (G, mu) with mu a 0-d float64 tensor on the host."""

    @staticmethod
    def forward(ctx, plan, h_k, sig_iw, n_target, mu_start):
        h_k = _c(h_k)
        sig = None if sig_iw is None else _c(sig_iw)
        g = _new((plan.r, plan.n_o, plan.n_o, plan.n_k), h_k)
        mu = plan.dyson_G(h_k, sig, g, n_target=n_target, mu=mu_start)
        ctx.save_for_backward(h_k, sig if sig is not None else torch.empty(0))
        ctx.args = (plan, n_target, mu, sig is not None)
        return g, torch.tensor(mu, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gg, gmu):
        h_k, sig = ctx.saved_tensors
        plan, n_target, mu, has_sig = ctx.args
        if gg is None:
            gg = torch.zeros((plan.r, plan.n_o, plan.n_o, plan.n_k), dtype=h_k.dtype, device=h_k.device)
        mubar = 0.0 if gmu is None else float(gmu)
        sb = _new((plan.r, plan.n_o, plan.n_o, plan.n_k), h_k)
        hb = torch.empty_like(h_k)
        plan.dyson_G_bwd(h_k, sig if has_sig else None, mu, _c(gg), sb, hb, n_target=n_target, mubar=mubar)
        return None, hb, (sb if has_sig else None), None, None


class Energy(torch.autograd.Function):
    """a14: Galitskii-Migdal total energy of (H0(k), Sigma_HF(k), Sigma^C(i w), G(i w)); a 0-d host tensor."""

    @staticmethod
    def forward(ctx, plan, h_k, shf_k, sig_iw, g_iw):
        h_k, shf_k, sig_iw, g_iw = _c(h_k), _c(shf_k), _c(sig_iw), _c(g_iw)
        e = plan.energy(h_k, shf_k, sig_iw, g_iw)[0]
        ctx.save_for_backward(h_k, shf_k, sig_iw, g_iw)
        ctx.plan = plan
        return torch.tensor(e, dtype=torch.float64)

    @staticmethod
    def backward(ctx, ge):
        h_k, shf_k, sig_iw, g_iw = ctx.saved_tensors
        hb, sb, cb, gb = (torch.empty_like(t) for t in (h_k, shf_k, sig_iw, g_iw))
        ctx.plan.energy_bwd(h_k, shf_k, sig_iw, g_iw, float(ge), hb, sb, cb, gb)
        return None, hb, sb, cb, gb


def energy(plan, H_k, shf_k, sig_iw, G_iw):
    return Energy.apply(plan, H_k, shf_k, sig_iw, G_iw)


# ----------------------------------------------------------------------------
# the iteration
# ----------------------------------------------------------------------------

def model_arrays(plan, H_R, V_R):
    """H0(k) = FT H0(R), V(q) = FT V(R) in the matrix layout (differentiable)."""
    H_k = FFT.apply(plan, qgw.R_TO_K, H_R)
    V_q = FFT.apply(plan, qgw.R_TO_K, V_R)
    return H_k, PairLayout.apply(plan, V_q)


def g0(plan, H_k, n_target):
    return DysonG.apply(plan, H_k, None, n_target, float("nan"))


def gw_iteration(plan, H_k, V_R, V_qm, G_iw, n_target, mu_start=float("nan")):
    """One GW iteration (mixing 1) from G(i w); returns (G, mu, Sigma^C(i w), Sigma_HF(k))."""
    no2 = plan.n_o * plan.n_o
    n_k = DLR.apply(plan, qgw.F_IW2BETA, G_iw, -1.0, 2)[0]
    n_R = FFT.apply(plan, qgw.K_TO_R, n_k)
    shf_k = FFT.apply(plan, qgw.R_TO_K, HartreeFock.apply(plan, V_R, n_R))
    Gt = FFT.apply(plan, qgw.K_TO_R, DLR.apply(plan, qgw.F_IW2TAU, G_iw, 1.0, 0))
    Gr = FFT.apply(plan, qgw.K_TO_R, DLR.apply(plan, qgw.F_IW2TAUR, G_iw, 1.0, 0))
    Pq = Bubble.apply(plan, Gt, Gr)
    Pnu = DLRPairs.apply(plan, qgw.B_TAU2IW, qgw.LAYOUT_SLAB, qgw.LAYOUT_MATRIX, Pq)
    Wc = DysonW.apply(plan, V_qm, Pnu)
    Wct = DLRPairs.apply(plan, qgw.B_IW2TAU, qgw.LAYOUT_MATRIX, qgw.LAYOUT_SLAB, Wc)
    Stk = Sigma.apply(plan, Gt, Wct)
    Siw = DLR.apply(plan, qgw.F_TAU2IW, Stk, 1.0, 1)
    Hs = Add.apply(plan, H_k, shf_k)
    G_new, mu = DysonG.apply(plan, Hs, Siw, n_target, mu_start)
    assert Siw.shape[1] * Siw.shape[2] == no2
    return G_new, mu, Siw, shf_k


def run(plan, H_R, V_R, n_target, n_iter=1, checkpointed=True):
    """n GW iterations from G0; returns the list of (G, mu, Sigma^C, Sigma_HF) per iteration."""
    H_k, V_qm = model_arrays(plan, H_R, V_R)
    G, mu = g0(plan, H_k, n_target)
    out = []
    for _ in range(n_iter):
        if checkpointed:
            res = checkpoint(gw_iteration, plan, H_k, V_R, V_qm, G, n_target, float(mu.detach()), use_reentrant=False)
        else:
            res = gw_iteration(plan, H_k, V_R, V_qm, G, n_target, float(mu.detach()))
        out.append(res)
        G, mu = res[0], res[1]
    return out



def backward_graph(groups):
    """One HIP graph holding the backward pass of many losses (many model instances in one launch).

    ``groups`` is a list of (stream, losses): each group's losses were built from the Functions above on its stream,
    without checkpointing (a checkpointed backward recomputes the forward, whose chemical-potential search reads its
    state back to the host). The capture runs on the first group's stream; the other streams are forked from it and
    joined back at the end, so the groups' adjoint chains run side by side, each group's in the order given. The
    forward's saved tensors are kept (``retain_graph``). The leaves' ``.grad`` must be None before the call; the
    gradients are then allocated from the graph's memory pool, and every ``replay()`` recomputes them into the same
    tensors from that forward. The replays read the forward's tensors at their addresses: keep the losses (and with
    them the forward's saved tensors) alive for as long as the graph is replayed.
    """
    s0 = groups[0][0]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s0):
        fork = torch.cuda.Event()
        fork.record(s0)
        for s, _ in groups[1:]:
            s.wait_event(fork)
        for s, losses in groups:
            if losses:
                with torch.cuda.stream(s):
                    torch.autograd.backward(losses, retain_graph=True)
        for s, _ in groups[1:]:
            s0.wait_stream(s)
    return g
