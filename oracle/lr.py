"""Oracle for the encrypted logistic-regression gradient step.

TEST INFRASTRUCTURE ONLY (see package docstring).

What is computed (paper Sec. 4): the linear-model gradient of eq. (obj)
linearised as in eq. (appr), sum_i y_i * p(y_i w.x_i) * x_i with the Table 2
polynomial p, followed by the update of eq. (update); Alg. 1 runs it on
encrypted data packed into blocks (Sec. 3, the packing of Han et al.).

Readings where the paper is silent (each listed in the design notes):
  * p approximates -L'(m) (Table 2's rows are positive at 0), so the step adds:
    w' = w + g,  g = (eta/n) sum_i p(m_i) z_i,  z_i = y_i x_i,  m_i = w.z_i.
  * packing: block b holds rows b*r .. b*r+r-1 of Z = y (.) X row-major, slot
    i*c + j = z_{b*r+i, j}; columns padded to c = 2^ceil(log2 d); W holds w in
    every row.
  * the per-block circuit is: u = Z (x) W; column sum by rotations 1..c/2;
    mask column 0; replicate by rotations -1..-c/2 (M holds m_i in row i);
    A = M^2, B3 = M * (a3 Z), B1 = M * (a1 Z); C = A * B3; B2 = A * (a2 Z)
    when a2 != 0 (Table 2's hinge row); G_b = C + a1-term + a0 Z (+ B2);
    cross-block sum; row sum by rotations c..(r/2)c.
  * a second packing, feature-major, puts z_{b*r+i, j} at slot j*r + i and w_j
    at every slot of feature block j.  A cyclic sum by rotations r..(c/2)r
    then leaves m_i in every feature block (no per-block mask or replicate);
    the polynomial runs on that directly, and after the cross-block sum the
    gradient is summed inside each feature block (rotations 1..r/2), masked to
    slot j*r and replicated by rotations -1..-r/2, once per step.
  * the margin sum may take baby and giant steps: with n_b baby steps, the
    worker keeps Rot(Z, b u) (b < n_b; u = r feature-major, 1 row-major) of
    its own data and rotates W by the same b u once per step, sums the n_b
    products Rot(Z, b u) (x) Rot(W, b u) as one degree-2 ciphertext (a
    rotation is a ring automorphism, so that is the sum of Rot(Z (x) W, b u)),
    relinearises and rescales it once, and finishes with the giant-step
    rotations n_b u .. (c/2) u.  Feature-major, the c/n_b giant steps g n_b r
    form a group of rotations (c r = N/2): for c/n_b <= 16 their sum
    x + sum_g Rot(x, g n_b r) is taken as one key switch, the rotations'
    inner products summed in Q u P before one ModDown (rotate_sum_hoisted).
  * the products C = A B3, B1 = M Z1 and B2 = A Z2 feed only additions, so
    they are formed at one level with one scale sC q (Z1's scale chosen for
    it), left unrelinearised and unrescaled, summed with the a0 term and across
    the blocks, and the sum is relinearised and rescaled once per step.
  * A = M^2 and B3 = M Z3 feed only those products, so they are rescaled but
    not relinearised (three components each): C is then of degree 4 in the
    secret (B2 of degree 3), and the step's one relinearisation switches d_2,
    d_3 and d_4 from s^2, s^3 and s^4 to s with three keys (rescaling a
    degree-2 ciphertext is the same per-component rounding; its error grows
    with s^2, a few bits below the scale here).
  * eta/n enters through the scale bookkeeping (an exact FP64 change of the
    declared scale), and W is brought to the gradient's scale by one integer
    multiplication and rescale, both fixed by plan_lr_step below.
"""
import math
from fractions import Fraction

import numpy as np

from . import ckks as O


# ---------------------------------------------------------------- plaintext reference
def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def ls_fit(f, bound, degree, nodes=400):
    """Least-squares polynomial fit of f on [-bound, bound] (eq. (3) with the
    sample points' uniform law taken to its continuous limit): minimise
    int (f - p)^2 dx over polynomials of the given degree.  Gram matrix of the
    monomials in closed form; right-hand side by Gauss-Legendre quadrature.
    Returns coefficients a_0..a_degree (lowest first)."""
    B = float(bound)
    G = np.zeros((degree + 1, degree + 1))
    for i in range(degree + 1):
        for j in range(degree + 1):
            k = i + j
            G[i, j] = 0.0 if k % 2 else 2.0 * B ** (k + 1) / (k + 1)
    x, w = np.polynomial.legendre.leggauss(nodes)
    x = x * B
    w = w * B
    fx = f(x)
    rhs = np.array([np.sum(w * fx * x ** i) for i in range(degree + 1)])
    return np.linalg.solve(G, rhs)


def grad_poly_binomial(bound=8.0):
    """Degree-3 least-squares fit of sigma(-m) = -L'(m) for the binomial
    deviance L(m) = log(1 + exp(-m)) (Table 1 / Table 2)."""
    return ls_fit(lambda x: sigmoid(-x), bound, 3)


def lr_gradient_fp64(X, y, w, coef, eta_over_n):
    """g = (eta/n) sum_i p(m_i) y_i x_i with m_i = y_i w.x_i (FP64); the step of
    eq. (update) with an L2 regulariser is w + g - eta lambda w."""
    z = y[:, None] * X
    m = z @ w
    p = coef[0] + coef[1] * m + coef[2] * m * m + coef[3] * m * m * m
    return eta_over_n * (p[:, None] * z).sum(axis=0)


# ---------------------------------------------------------------- packing
def pack_blocks(X, y, S):
    """Row-major block packing of Z = y (.) X.  Returns (blocks [B][S] float64, c, r)."""
    n, d = X.shape
    c = 1 << max(0, math.ceil(math.log2(d)))
    r = S // c
    B = (n + r - 1) // r
    Z = np.zeros((B * r, c))
    Z[:n, :d] = y[:, None] * X
    return Z.reshape(B, r * c), c, r


def pack_weights(w, S, c):
    v = np.zeros(c)
    v[: w.shape[0]] = w
    return np.tile(v, S // c)


def column_mask(S, c):
    m = np.zeros(S)
    m[::c] = 1.0
    return m


ROWS, FEATURES = 0, 1  # the two block layouts


def pack_blocks_features(X, y, S):
    """Feature-major packing: slot j*r + i of block b = z_{b*r+i, j}."""
    blocks, c, r = pack_blocks(X, y, S)
    return np.ascontiguousarray(blocks.reshape(-1, r, c).transpose(0, 2, 1).reshape(-1, S)), c, r


def pack_weights_features(w, S, c):
    v = np.zeros(c)
    v[: w.shape[0]] = w
    return np.repeat(v, S // c)


def feature_mask(S, r):
    """1 at the first slot of every feature block (slots j*r)."""
    m = np.zeros(S)
    m[::r] = 1.0
    return m


# ---------------------------------------------------------------- scale plan
class ScaleError(ValueError):
    pass


class LevelError(ValueError):
    pass


def llround(x):
    """C llround: nearest integer, halves away from zero (exact on FP64)."""
    fx = Fraction(x)
    fl = math.floor(fx)
    fr = fx - fl
    if fr > Fraction(1, 2) or (fr == Fraction(1, 2) and fx > 0):
        fl += 1
    return int(fl)


K_MAX = 2 ** 62


def term_scale(coef, q0, eta_over_n, fm_cap=None):
    """Target scale T of the gradient terms, a power of two.  The output g has
    scale s_g = T / (eta/n) and must keep 10 bits of headroom below q_0 (the
    last limb of the chain): T is the largest power of two with
    T / (eta/n) <= 2^(floor(log2 q_0) - 10), kept between the powers of two
    with T * min(|a1|, |a2|, |a3|) in [2^22, 2^23) (coefficient resolution)
    and in [2^30, 2^31).  The rescale noise of the terms is fixed in size,
    so a larger T makes the terms relatively more precise.
    fm_cap (feature-major): a further upper bound that keeps the gradient
    mask's plaintext scale at 2^34 or more; a layout that cannot meet it
    together with the lower bound is refused."""
    nz = [abs(a) for a in (coef[1], coef[2], coef[3]) if a != 0.0]
    if not nz:
        raise ScaleError("polynomial needs a nonzero a1, a2 or a3")
    _, e = math.frexp(min(nz))
    lo = math.ldexp(1.0, 23 - e)
    hi = math.ldexp(1.0, 31 - e)
    _, ec = math.frexp(math.ldexp(eta_over_n, int(q0).bit_length() - 1 - 10))
    cap = math.ldexp(1.0, ec - 1)
    if fm_cap is not None:
        t = min(hi, cap, fm_cap)
        if t < lo:
            raise ScaleError("feature-major step: the gradient mask would fall below scale 2^34 "
                             "(data scale too small for n/eta); use the row-major layout")
        return t
    return max(lo, min(hi, cap))


def plan_lr_step(q, level, s_Z, s_W, coef, eta_over_n, w_decay=0.0, layout=ROWS):
    """FP64 scale schedule of one gradient step at W's level `level`.
    Every expression is evaluated left to right exactly as written.
    w_decay = eta * lambda of an L2 regulariser R = lambda/2 |w|^2 (eq. (obj)):
    its gradient step -eta lambda w is folded into W's renormalisation."""
    if level < 4:
        raise LevelError("a gradient step needs 4 levels; W is at level %d" % level)
    if not (0.0 <= w_decay < 1.0):
        raise ScaleError("w_decay must lie in [0, 1)")
    if layout == FEATURES:
        return _plan_features(q, level, s_Z, s_W, coef, eta_over_n, w_decay)
    ql = float(q[level])
    ql1 = float(q[level - 1])
    ql2 = float(q[level - 2])
    ql3 = float(q[level - 3])
    s1 = s_Z * s_W / ql
    s_mask = ql2 * ql1 / s1
    sM = s1 * s_mask / ql1
    sA = sM * sM / ql2
    T = term_scale(coef, q[0], eta_over_n)
    sZ3 = T * ql3 / sA * ql2 / sM
    k3 = llround(coef[3] * sZ3 * ql1 / s_Z)
    sB3 = sM * sZ3 / ql2
    sC = sA * sB3 / ql3
    sZ1 = sC * ql3 / sM
    k1 = llround(coef[1] * sZ1 * ql2 / s_Z)
    sB1 = sM * sZ1
    kB1 = 0
    k0 = llround(coef[0] * sC * ql3 / s_Z)
    sZ2 = sC * ql3 / sA
    k2 = llround(coef[2] * sZ2 * ql2 / s_Z)
    s_g = sC / eta_over_n
    kW = llround((1.0 - w_decay) * s_g * ql3 / s_W)
    for name, k in (("k0", k0), ("k1", k1), ("k2", k2), ("k3", k3), ("kB1", kB1), ("kW", kW)):
        if abs(k) >= K_MAX:
            raise ScaleError("%s = %d out of range" % (name, k))
    return dict(level=level, s1=s1, s_mask=s_mask, sM=sM, sA=sA, T=T, sZ3=sZ3, k3=k3, sB3=sB3,
                sC=sC, sZ1=sZ1, k1=k1, sB1=sB1, kB1=kB1, k0=k0, sZ2=sZ2, k2=k2, s_g=s_g, kW=kW,
                level_out=level - 4, s_gsum=s_g, layout=ROWS)


def _plan_features(q, level, s_Z, s_W, coef, eta_over_n, w_decay):
    """Feature-major schedule: M = u at level l-1 (no mask), the polynomial
    one level higher than in the row-major circuit, the gradient summed at
    level l-3 and masked down to level l-4.  The mask's plaintext scale
    returns W' (and g) to the data's scale s_Z, so that M's scale at the next
    step stays near q and every integer constant keeps its resolution."""
    ql = float(q[level])
    ql1 = float(q[level - 1])
    ql2 = float(q[level - 2])
    ql3 = float(q[level - 3])
    _, ef = math.frexp(s_Z * ql3 * eta_over_n)
    T = term_scale(coef, q[0], eta_over_n, math.ldexp(1.0, ef - 1 - 34))
    s1 = s_Z * s_W / ql
    sM = s1
    sA = sM * sM / ql1
    sZ3 = T * ql2 / sA * ql1 / sM
    k3 = llround(coef[3] * sZ3 * ql / s_Z)
    sB3 = sM * sZ3 / ql1
    sC = sA * sB3 / ql2
    sZ1 = sC * ql2 / sM
    k1 = llround(coef[1] * sZ1 * ql1 / s_Z)
    sB1 = sM * sZ1
    kB1 = 0
    k0 = llround(coef[0] * sC * ql2 / s_Z)
    sZ2 = sC * ql2 / sA
    k2 = llround(coef[2] * sZ2 * ql1 / s_Z)
    s_gsum = sC / eta_over_n
    s_mask = s_Z * ql3 / s_gsum
    s_g = s_gsum * s_mask / ql3
    kW = llround((1.0 - w_decay) * s_g * ql3 / s_W)
    for name, k in (("k0", k0), ("k1", k1), ("k2", k2), ("k3", k3), ("kB1", kB1), ("kW", kW)):
        if abs(k) >= K_MAX:
            raise ScaleError("%s = %d out of range" % (name, k))
    return dict(level=level, s1=s1, s_mask=s_mask, sM=sM, sA=sA, T=T, sZ3=sZ3, k3=k3, sB3=sB3,
                sC=sC, sZ1=sZ1, k1=k1, sB1=sB1, kB1=kB1, k0=k0, sZ2=sZ2, k2=k2, s_g=s_g, kW=kW,
                level_out=level - 4, s_gsum=s_gsum, layout=FEATURES)


GIANT_MAX = 16  # most giant steps (c / n_baby) a hoisted feature-major giant sum takes


def giant_hoisted(c, layout, n_baby):
    """Feature-major margins with baby steps take their giant steps as one
    hoisted sum: the rotations by g n_baby r (g < c / n_baby) are a group
    (c r = N/2), so their sum is x + sum_g Rot(x, g n_baby r), one key switch
    with every rotation's inner product summed before one ModDown."""
    return layout == FEATURES and 1 < n_baby < c and c // n_baby <= GIANT_MAX


def slot_sum_groups(r):
    """Reading 28: every sum of the rotations by 0, u, 2u, .., (r - 1) u
    (r = 2^k; the margin, column, row and feature-block slot sums and the
    replications) is taken as one hoisted sum per group of index bits, the
    rotations of a group scaled by u.  The k bits split into
    ceil(k / 3) groups whose sizes differ by at most one, the smaller
    groups on the low bits; a group of s bits starting at bit b contributes
    the rotations j * 2^b for j = 1 .. 2^s - 1.  Summing over every group in
    turn covers each index i < r exactly once (its base-2^s digits)."""
    k = 0
    while (1 << k) < r:
        k += 1
    groups = []
    if k == 0:
        return groups
    ng = -(-k // 3)
    sizes = [k // ng] * ng
    for i in range(k % ng):
        sizes[ng - 1 - i] += 1
    b = 0
    for s in sizes:
        groups.append([j * (1 << b) for j in range(1, 1 << s)])
        b += s
    return groups


def rotation_steps(c, r, layout=ROWS, n_baby=1):
    """Rotation steps used by the step (reading 28 for the slot sums).
    Row-major: the baby steps b < n_baby, n_baby * t for the steps t of
    slot_sum_groups(c / n_baby) (the column sum), -t for those of
    slot_sum_groups(c) (the replication), c * t for those of
    slot_sum_groups(r) (the row sum).  Feature-major: the baby steps b r
    (b < n_baby), the giant steps g n_baby r (g < c / n_baby) when hoisted,
    else n_baby r t for the steps t of slot_sum_groups(c / n_baby), and +-t
    for those of slot_sum_groups(r).  With n_baby = 1 the set also holds the
    margins of lr_margins / lr_infer in the same layout."""
    nb = max(n_baby, 1)
    if layout == FEATURES:
        st = set(b * r for b in range(1, nb))
        if giant_hoisted(c, layout, nb):
            st.update(g * nb * r for g in range(1, c // nb))
        else:
            st.update(nb * r * t for grp in slot_sum_groups(c // nb) for t in grp)
        st.update(s * t for grp in slot_sum_groups(r) for t in grp for s in (1, -1))
        return sorted(st)
    st = set(b for b in range(1, nb))
    for grp in slot_sum_groups(c // nb):
        st.update(nb * t for t in grp)
    for grp in slot_sum_groups(c):
        st.update(-t for t in grp)
    for grp in slot_sum_groups(r):
        st.update(c * t for t in grp)
    return sorted(st)


# ---------------------------------------------------------------- encrypted step
def lr_grad_step(P, keys, Z, W, mask_m, coef, eta_over_n, c, r, plan=None, w_decay=0.0, layout=ROWS, Zrot=None,
                 n_baby=1):
    """One step of eq. (appr) + eq. (update) on ciphertexts (coefficient form).
    Z: list of block ciphertexts (same level >= W.level, same scale);
    W: weight ciphertext; mask_m: integer plaintext of column_mask at scale
    plan['s_mask'].  n_baby > 1 takes the margins by baby and giant steps,
    with Zrot = rotate_data(P, keys, Z, u, n_baby) (u = r feature-major, 1
    row-major).
    Returns (W', g); g excludes the regulariser's -eta lambda w."""
    l = W.level
    pl = plan or plan_lr_step(P.q, l, Z[0].scale, W.scale, coef, eta_over_n, w_decay, layout)
    if layout == FEATURES:
        return _step_features(P, keys, Z, W, mask_m, c, r, pl, Zrot, n_baby)
    G = None
    if n_baby > 1:
        Ws = [W] + [O.rotate(P, W, b, keys) for b in range(1, n_baby)]
    for k, zb in enumerate(Z):
        if n_baby > 1:
            u = _margin_products(P, keys, [zb] + list(Zrot[k]), Ws, l, pl["s1"])
            t = n_baby
        else:
            u = O.rescale(P, O.mul(P, O.drop(zb, l), W, keys), scale=pl["s1"])
            t = 1
        for grp in slot_sum_groups(c // t):  # column sum (reading 28)
            u = O.rotate_sum_hoisted(P, u, [t * s for s in grp], keys)
        M = O.rescale(P, O.mul_plain(P, u, mask_m, pl["s_mask"]), scale=pl["sM"])
        for grp in slot_sum_groups(c):  # replicate column 0 over the row
            M = O.rotate_sum_hoisted(P, M, [-s for s in grp], keys)
        A = _rs_product(P, M, M)
        Z3 = O.rescale(P, O.mul_int(P, O.drop(zb, l - 1), pl["k3"]), scale=pl["sZ3"])
        B3 = _rs_product(P, M, Z3)
        Z1 = O.rescale(P, O.mul_int(P, O.drop(zb, l - 2), pl["k1"]), scale=pl["sZ1"])
        Z2 = None
        if pl["k2"] != 0:
            Z2 = O.rescale(P, O.mul_int(P, O.drop(zb, l - 2), pl["k2"]), scale=pl["sZ2"])
        Gb = _terms_prescale(P, zb, A, B3, M, Z1, Z2, l - 3, pl)
        G = Gb if G is None else O.add_n(P, l - 3, G, Gb)
    # one relinearisation and one rescale of the summed terms
    G = O.rescale(P, O.relin_n(P, G, pl["sC"] * float(P.q[l - 3]), l - 3, keys), scale=pl["sC"])
    for grp in slot_sum_groups(r):  # row sum
        G = O.rotate_sum_hoisted(P, G, [c * s for s in grp], keys)
    g = O.CT(G.data, G.level, pl["s_g"])
    Wn = O.rescale(P, O.mul_int(P, O.drop(W, l - 3), pl["kW"]), scale=pl["s_g"])
    return O.add(P, Wn, g), g


def _rs_product(P, x, y):
    """RS(x (x) y), not relinearised: a degree-2 array [3][l][N] one level
    below x and y (which share their level)."""
    l = x.level
    return O.rescale_n(P, l, O.tensor_n(P, l, x.data, y.data))


def _terms_prescale(P, zb, A, B3, M, Z1, Z2, lp, pl):
    """The block's gradient terms, unrescaled, as one degree-4 array at level lp
    with scale sC q_lp: C = A (x) B3 (A, B3 of degree 2), B1 = M (x) Z1 (M
    dropped to lp; Z1 carries sC q_lp / sM), k0 Z, and for a2 != 0
    B2 = A (x) Z2."""
    G = O.add_n(P, lp, O.tensor_n(P, lp, A, B3), O.tensor_n(P, lp, O.drop(M, lp).data, Z1.data))
    G = O.add_n(P, lp, G, O.mul_int(P, O.drop(zb, lp), pl["k0"]).data)
    if pl["k2"] != 0:
        G = O.add_n(P, lp, G, O.tensor_n(P, lp, A, Z2.data))
    return G


def rotate_data(P, keys, Z, unit, n_baby):
    """The worker's baby-step copies of its data: Rot(z_b, b unit) for
    b = 1 .. n_baby - 1, per block (unit = r feature-major, 1 row-major)."""
    return [[O.rotate(P, zb, b * unit, keys) for b in range(1, n_baby)] for zb in Z]


def _margin_products(P, keys, zs, Ws, l, s1):
    """RS(relin(sum_b zs[b] (x) Ws[b])) at scale s1: the baby-step sum of the
    products, one degree-2 ciphertext relinearised and rescaled once."""
    D = None
    for zr, wr in zip(zs, Ws):
        t3 = O.tensor(P, O.drop(zr, l), wr)[0]
        D = t3 if D is None else O.add_n(P, l, D, t3)
    return O.rescale(P, O.relin(P, D, s1 * float(P.q[l]), l, keys), scale=s1)


def _step_features(P, keys, Z, W, mask_m, c, r, pl, Zrot=None, n_baby=1):
    """Feature-major step; mask_m: integer plaintext of feature_mask at scale
    plan['s_mask'] (used at level l-3)."""
    l = W.level
    G = None
    if n_baby > 1:
        Ws = [W] + [O.rotate(P, W, b * r, keys) for b in range(1, n_baby)]
    for k, zb in enumerate(Z):
        if n_baby > 1:
            u = _margin_products(P, keys, [zb] + list(Zrot[k]), Ws, l, pl["s1"])
            t = n_baby
        else:
            u = O.rescale(P, O.mul(P, O.drop(zb, l), W, keys), scale=pl["s1"])
            t = 1
        if giant_hoisted(c, FEATURES, n_baby):  # margins: the giant steps as one key switch
            u = O.rotate_sum_hoisted(P, u, [g * n_baby * r for g in range(1, c // n_baby)], keys)
        else:  # margins: cyclic sum over the feature blocks t r, 2 t r, .., grouped (reading 28)
            for grp in slot_sum_groups(c // t):
                u = O.rotate_sum_hoisted(P, u, [t * r * s for s in grp], keys)
        M = u
        A = _rs_product(P, M, M)
        Z3 = O.rescale(P, O.mul_int(P, O.drop(zb, l), pl["k3"]), scale=pl["sZ3"])
        B3 = _rs_product(P, M, Z3)
        Z1 = O.rescale(P, O.mul_int(P, O.drop(zb, l - 1), pl["k1"]), scale=pl["sZ1"])
        Z2 = None
        if pl["k2"] != 0:
            Z2 = O.rescale(P, O.mul_int(P, O.drop(zb, l - 1), pl["k2"]), scale=pl["sZ2"])
        Gb = _terms_prescale(P, zb, A, B3, M, Z1, Z2, l - 2, pl)
        G = Gb if G is None else O.add_n(P, l - 2, G, Gb)
    # one relinearisation and one rescale of the summed terms
    G = O.rescale(P, O.relin_n(P, G, pl["sC"] * float(P.q[l - 2]), l - 2, keys), scale=pl["sC"])
    for grp in slot_sum_groups(r):  # sum over the samples inside each feature block (reading 28)
        G = O.rotate_sum_hoisted(P, G, grp, keys)
    G = O.CT(G.data, G.level, pl["s_gsum"])
    g = O.rescale(P, O.mul_plain(P, G, mask_m, pl["s_mask"]), scale=pl["s_g"])
    for grp in slot_sum_groups(r):  # replicate g_j over its feature block
        g = O.rotate_sum_hoisted(P, g, [-t for t in grp], keys)
    Wn = O.rescale(P, O.mul_int(P, O.drop(W, l - 3), pl["kW"]), scale=pl["s_g"])
    return O.add(P, Wn, g), g


# ---------------------------------------------------------------- paper-order circuit
def lr_grad_step_plain(P, keys, Z, W, mask_m, coef, eta_over_n, c, r, plan=None, w_decay=0.0, layout=ROWS):
    """The same step in the order Sec. 3 and Sec. 4 state it, with none of the
    fused schedule above: every ciphertext product is relinearised and rescaled
    before it is used (Sec. 3, multiplication then scaling), every slot sum is
    a sequence of rotate-and-adds, each block's gradient terms C, B1, k0 Z
    (and B2) are rescaled on their own before the cross-block sum of
    eq. (appr), and W is updated by eq. (update).  No baby steps, no hoisted
    key switch, no degree-3 or degree-4 ciphertext, no unrescaled sum.

    It takes the same scale plan (plan_lr_step) as lr_grad_step: every term
    still lands on the plan's scale sC, so the two circuits compute the same
    slots and differ only by where they round (rescale and key-switch noise).
    It is the reference lr_grad_step is pinned against.  Returns (W', g)."""
    l = W.level
    pl = plan or plan_lr_step(P.q, l, Z[0].scale, W.scale, coef, eta_over_n, w_decay, layout)
    feat = layout == FEATURES
    lt = l - 2 if feat else l - 3  # level of the products C, B1 (and B2) before their rescale
    G = None
    for zb in Z:
        u = O.rescale(P, O.mul(P, O.drop(zb, l), W, keys), scale=pl["s1"])
        t = 1
        while t < c:  # margins: rotate-and-add over the columns (row-major) or feature blocks
            u = O.add(P, u, O.rotate(P, u, t * r if feat else t, keys))
            t *= 2
        if feat:
            M = u
        else:
            M = O.rescale(P, O.mul_plain(P, u, mask_m, pl["s_mask"]), scale=pl["sM"])
            t = 1
            while t < c:  # replicate m_i over row i
                M = O.add(P, M, O.rotate(P, M, -t, keys))
                t *= 2
        lm = M.level  # l-1 feature-major, l-2 row-major
        A = O.rescale(P, O.mul(P, M, M, keys), scale=pl["sA"])
        Z3 = O.rescale(P, O.mul_int(P, O.drop(zb, lm + 1), pl["k3"]), scale=pl["sZ3"])
        B3 = O.rescale(P, O.mul(P, M, Z3, keys), scale=pl["sB3"])
        C = O.rescale(P, O.mul(P, A, B3, keys), scale=pl["sC"])
        Z1 = O.rescale(P, O.mul_int(P, O.drop(zb, lt + 1), pl["k1"]), scale=pl["sZ1"])
        B1 = O.rescale(P, O.mul(P, O.drop(M, lt), Z1, keys), scale=pl["sC"])
        Z0 = O.rescale(P, O.mul_int(P, O.drop(zb, lt), pl["k0"]), scale=pl["sC"])
        Gb = O.add(P, O.add(P, C, B1), Z0)
        if pl["k2"] != 0:
            Z2 = O.rescale(P, O.mul_int(P, O.drop(zb, lt + 1), pl["k2"]), scale=pl["sZ2"])
            Gb = O.add(P, Gb, O.rescale(P, O.mul(P, A, Z2, keys), scale=pl["sC"]))
        G = Gb if G is None else O.add(P, G, Gb)
    if feat:
        t = 1
        while t < r:  # sum over the samples inside each feature block
            G = O.add(P, G, O.rotate(P, G, t, keys))
            t *= 2
        G = O.CT(G.data, G.level, pl["s_gsum"])
        g = O.rescale(P, O.mul_plain(P, G, mask_m, pl["s_mask"]), scale=pl["s_g"])
        t = 1
        while t < r:  # replicate g_j over its feature block
            g = O.add(P, g, O.rotate(P, g, -t, keys))
            t *= 2
    else:
        t = 1
        while t < r:  # sum over the rows, replicated in every row
            G = O.add(P, G, O.rotate(P, G, t * c, keys))
            t *= 2
        g = O.CT(G.data, G.level, pl["s_g"])
    Wn = O.rescale(P, O.mul_int(P, O.drop(W, l - 3), pl["kW"]), scale=pl["s_g"])
    return O.add(P, Wn, g), g


# ---------------------------------------------------------------- encrypted inference
def lr_margins(P, keys, Z, W, c, r, layout=ROWS):
    """The margins m_i = w.z_i per block (eq. (appr)'s inner products):
    u = RS(relin(Z (x) W)), then the sum of Rot(u, j unit) over j < c (unit
    = r feature-major, 1 row-major) as grouped hoisted sums (reading 28)."""
    l = W.level
    unit = r if layout == FEATURES else 1
    out = []
    for zb in Z:
        u = O.rescale(P, O.mul(P, O.drop(zb, l), W, keys))
        for grp in slot_sum_groups(c):
            u = O.rotate_sum_hoisted(P, u, [unit * s for s in grp], keys)
        out.append(u)
    return out


def plan_lr_infer(q, level, s_Z, s_W, coef):
    """FP64 schedule of p(u) on the margins u (level l-1, scale s_u):
    U2 = RS(relin(u u)), H = RS(k3 u) + k2c, p = RS(relin(H U2)) + RS(k1 u) +
    k0c at level l-3 and scale s_p = s_u.  Expressions evaluated left to right
    exactly as written."""
    if level < 3:
        raise LevelError("inference with the polynomial needs 3 levels; W is at level %d" % level)
    ql, q1, q2 = float(q[level]), float(q[level - 1]), float(q[level - 2])
    s_u = s_Z * s_W / ql
    s_u2 = s_u * s_u / q1
    s_p = s_u
    s_h = s_p * q2 / s_u2
    k3 = coef[3] * s_h * q1 / s_u
    k2c = coef[2] * s_h
    k1 = coef[1] * s_p * q2 / s_u
    k0c = coef[0] * s_p
    for name, k in (("k3", k3), ("k2c", k2c), ("k1", k1), ("k0c", k0c)):
        if not abs(k) < K_MAX:
            raise ScaleError("%s out of range" % name)
    return dict(level=level, level_out=level - 3, s_u=s_u, s_u2=s_u2, s_h=s_h, s_p=s_p, k3=llround(k3),
                k2c=llround(k2c), k1=llround(k1), k0c=llround(k0c))


def lr_infer(P, keys, Z, W, c, r, layout=ROWS, coef=None):
    """Encrypted scoring: the margins, and with coef the polynomial
    p(m) = a0 + a1 m + a2 m^2 + a3 m^3 slot by slot (Table 2's p approximates
    -L'; for the binomial deviance p(m) ~ sigma(-m))."""
    us = lr_margins(P, keys, Z, W, c, r, layout)
    if coef is None:
        return us
    pl = plan_lr_infer(P.q, W.level, Z[0].scale, W.scale, coef)
    out = []
    for u in us:
        U2 = O.rescale(P, O.mul(P, u, u, keys))
        H = O.add_const(P, O.rescale(P, O.mul_int(P, u, pl["k3"]), scale=pl["s_h"]), pl["k2c"])
        T = O.rescale(P, O.mul(P, H, U2, keys), scale=pl["s_p"])
        L = O.rescale(P, O.mul_int(P, O.drop(u, u.level - 1), pl["k1"]), scale=pl["s_p"])
        out.append(O.add_const(P, O.add(P, T, L), pl["k0c"]))
    return out
