"""Worker / parameter-server loop of the paper over the C ABI.

Alg. 2 (parameter server): generates the keys, encrypts the data blocks and
the initial weights with sk, and on a worker's request decrypts the
weights, takes them as its own copy and sends them back freshly encrypted at
the top level.  Alg. 1 (worker): evaluates eq. (appr) + eq. (update)
homomorphically once per iteration and requests a refresh every `l`
iterations.  On one GPU both roles share the device; the request is a host
call (the paper's MPI messages carry one ciphertext each way).
"""
import numpy as np

from . import he as H


class ParameterServer:
    """Holds sk (inside `keys`) and the plaintext weights; Alg. 2."""

    def __init__(self, ctx, keys, d, cols, seed_enc, first_index=1 << 24, layout=H.LAYOUT_ROWS):
        self.ctx, self.keys, self.d, self.cols, self.layout = ctx, keys, d, cols, layout
        self.seed_enc = seed_enc
        self.index = first_index  # ChaCha20 stream index of the next weight encryption
        self.w = None
        self._buf = None
        self._pt = None

    def encrypt_weights(self, w):
        """Encrypt w at the top level into the server's one weight buffer."""
        ctx = self.ctx
        L = ctx.n_q - 1
        self.w = np.array(w, dtype=np.float64)
        m = ctx.encode(H.pack_weights(self.w, ctx.S, self.cols, self.layout), ctx.delta)
        if self._buf is None:
            self._buf = ctx.ct_empty(L)
            self._pt = ctx.pt_empty(L)
        ct = ctx.encrypt(ctx.pt_load(m, L, ctx.delta, out=self._pt), self.keys, self.seed_enc, self.index,
                         out=self._buf)
        self.index += 1
        return ct

    def refresh(self, W):
        """Decrypt the worker's weights, update the server's copy, re-encrypt."""
        slots = self.ctx.decrypt_decode(W, self.keys).real
        return self.encrypt_weights(H.unpack_weights(slots, self.cols, self.d, self.layout))


class Worker:
    """Evaluates the encrypted gradient step on its shard; Alg. 1."""

    TERMS_KEPT = 8  # (level, scale) pairs whose data terms the worker keeps

    def __init__(self, ctx, keys, Z, coef, eta_over_n, cols, rows, mode=2, w_decay=0.0, layout=H.LAYOUT_ROWS,
                 n_baby=1, Zrot=None, terms=True):
        """n_baby > 1: the worker keeps the baby-step rotations
        of its data (n_baby - 1 copies of the shard), computed here unless
        given as Zrot (ctx.rotate_data).  terms: the worker keeps the step's
        data terms (ctx.lr_data_terms) per weight level and scale, computed
        on first use; the weights return to the same levels and scales every
        refresh period."""
        self.ctx, self.keys, self.Z = ctx, keys, Z
        self.coef, self.eta_over_n, self.w_decay = list(coef), eta_over_n, w_decay
        self.cols, self.rows, self.mode, self.layout = cols, rows, mode, layout
        self.n_baby = n_baby
        if n_baby > 1 and Zrot is None:
            Zrot = ctx.rotate_data(Z, H.baby_unit(layout, rows), n_baby, keys)
        self.Zrot = Zrot if n_baby > 1 else None
        # argument arrays built once: the blocks and their copies do not move
        self._za = H.ct_array(Z)
        self._zra = H.ct_array(self.Zrot) if self.Zrot else None
        self._masks = {}
        self._bufs = {}
        self.terms = terms
        self._terms = {}

    def _mask(self, level, s_mask):
        key = (level, s_mask)
        if key not in self._masks:
            ctx = self.ctx
            m = ctx.encode(H.step_mask(ctx.S, self.cols, self.layout), s_mask)
            self._masks[key] = ctx.pt_load(m, H.mask_level(level, self.layout), s_mask)
        return self._masks[key]

    def _out(self, level, slot):
        key = (level, slot)
        if key not in self._bufs:
            self._bufs[key] = self.ctx.ct_empty(level)
        return self._bufs[key]

    def step(self, W, want_g=False):
        """One iteration; the output lives in a buffer owned per output level
        (levels only decrease between refreshes, so it never aliases W)."""
        ctx = self.ctx
        pl = ctx.plan_lr_step(W.level, self.Z[0].scale, W.scale, self.coef, self.eta_over_n, self.w_decay,
                              self.layout)
        mask = self._mask(W.level, pl["s_mask"])
        zk = None
        if self.terms:
            key = (W.level, W.scale)
            if key not in self._terms:
                if len(self._terms) >= self.TERMS_KEPT:
                    self._terms.pop(next(iter(self._terms)))
                cts = ctx.lr_data_terms(self.Z, W.level, W.scale, self.coef, self.eta_over_n, self.w_decay,
                                        self.layout)
                self._terms[key] = (cts, H.ct_array(cts))
            zk = self._terms[key][1]
        lo = W.level - 4
        W_out = self._out(lo, 0)
        G_out = self._out(lo, 1) if want_g else None
        return ctx.lr_grad_step(self._za, W, mask, self.coef, self.eta_over_n, self.cols, self.rows, self.keys,
                                mode=self.mode, W_out=W_out, G_out=G_out, want_g=want_g, w_decay=self.w_decay,
                                layout=self.layout, Zrot=self._zra, n_baby=self.n_baby, Zk=zk)


def encrypt_shard(ctx, keys, X, y, seed_enc, layout=H.LAYOUT_ROWS):
    """Alg. 2 initialisation: pack Z = y (.) X into blocks and encrypt each with sk."""
    blocks, cols, rows = H.pack_blocks(X, y, ctx.S, layout)
    L = ctx.n_q - 1
    Z = ctx.ct_block(blocks.shape[0], L)
    for i in range(blocks.shape[0]):
        ctx.encrypt(ctx.pt_load(ctx.encode(blocks[i], ctx.delta), L, ctx.delta), keys, seed_enc, i, out=Z[i])
    return Z, cols, rows


def train(ctx, keys, X, y, coef, eta, iterations, refresh_every, w0, seed_enc, mode=2, record=None, l2=0.0,
          layout=H.LAYOUT_ROWS, n_baby=1):
    """Alg. 1 + Alg. 2 on one GPU.  Returns the server's final plaintext
    weights (after a last refresh) and, if `record` is a list, appends the
    decrypted weights after every iteration.  l2: lambda of R = lambda/2 |w|^2."""
    n, d = X.shape
    Z, cols, rows = encrypt_shard(ctx, keys, X, y, seed_enc, layout)
    ps = ParameterServer(ctx, keys, d, cols, seed_enc, layout=layout)
    worker = Worker(ctx, keys, Z, coef, eta / n, cols, rows, mode=mode, w_decay=eta * l2, layout=layout,
                    n_baby=n_baby)
    W = ps.encrypt_weights(w0)
    for k in range(1, iterations + 1):
        W, _ = worker.step(W)
        if record is not None:
            record.append(H.unpack_weights(ctx.decrypt_decode(W, keys).real, cols, d, layout).copy())
        if k % refresh_every == 0 or W.level < 4:
            W = ps.refresh(W)
    ps.refresh(W)
    return ps.w
