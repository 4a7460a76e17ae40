"""Agreement rule for PCG iteration counts shared by the GPU parity tests."""


def iters_agree(gpu_iters, oinfo, tol, bnorm):
    """Equal counts; or one apart where the oracle's deciding residual lies
    within a factor 1.2 of the threshold on the side that makes the
    difference (just above it one iteration before the oracle stopped, or just
    below it where the oracle stopped)."""
    if gpu_iters == oinfo.iters:
        return True
    if abs(gpu_iters - oinfo.iters) != 1:
        return False
    thr = tol * bnorm
    if gpu_iters < oinfo.iters:
        return oinfo.resnorms[gpu_iters] <= 1.2 * thr
    return oinfo.resnorms[oinfo.iters] >= thr / 1.2
