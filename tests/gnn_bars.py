"""Bars of the learned proposal's GPU-vs-oracle checks (tests/test_gpu_gnn.py).

The device keeps messages, activations and dZ in BF16 and accumulates in FP32;
the oracle is FP64.  The bars below are derived from the BF16 storage-point
model (tests/gnn_bf16_model.py) run on the same inputs as the GPU tests: over
three problems, five parameter seeds and six FP32-order jitters of 3e-7 the
model reaches logit errors of 0.017, loss errors of 0.0084, whole-gradient
cosines down to 0.9953 and relative L2 errors up to 0.097, per-tensor
relative L2 errors up to 0.147 and per-tensor norm ratios within
[0.950, 1.059].  Each bar leaves at least 1.5x that spread
(tests/test_gnn_bars.py checks this on the CPU) while a gradient tensor scaled
by 2 (relative error 1, norm ratio 2) fails the per-tensor bars.
"""
LOGIT_REL = 3e-2          # max |logit - ref| / max(1, |ref|_inf)
LOSS_REL = 2e-2           # |loss - ref| / max(1, |ref|)
GRAD_COS_MIN = 0.99       # cosine of the whole gradient vector
GRAD_REL_MAX = 0.15       # relative L2 error of the whole gradient
TENSOR_REL_MAX = 0.3      # relative L2 error of each parameter tensor
TENSOR_RATIO = (0.85, 1.15)   # |g_k| / |g_ref_k| of each parameter tensor
TENSOR_MIN_NORM = 1e-7    # tensors with a smaller reference norm: |g_k| <= 1e-5 instead


def check(c):
    """Assert the bars on the output of gnn_bf16_model.compare (or the same
    quantities measured on the GPU).  Returns the list of failed bars."""
    bad = []
    if c["logit"] > LOGIT_REL:
        bad.append(("logit", c["logit"]))
    if c["loss"] > LOSS_REL:
        bad.append(("loss", c["loss"]))
    if c["cos"] < GRAD_COS_MIN:
        bad.append(("cos", c["cos"]))
    if c["rel"] > GRAD_REL_MAX:
        bad.append(("rel", c["rel"]))
    for k, v in c["tensor_rel"].items():
        if v is None:
            continue
        if v > TENSOR_REL_MAX:
            bad.append((k + ":rel", v))
        r = c["tensor_ratio"][k]
        if not (TENSOR_RATIO[0] <= r <= TENSOR_RATIO[1]):
            bad.append((k + ":ratio", r))
    return bad
