"""The BF16 stochastic rounding's step term, on the host (no GPU): an emulation of the kernels'
rounding (16 hash bits added below the kept mantissa, then truncation; the hash is the
MurmurHash3 32-bit finalizer of node, direction with the step term above its five bits, and the
value) applied to a population that gains a constant fraction of an ulp every step."""
import numpy as np

M32 = 0xFFFFFFFF


def fmix32(h):
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & M32
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & M32
    h ^= h >> 16
    return h


def bf16_sr(v: float, node: int, d: int) -> float:
    u = int(np.float32(v).view(np.uint32))
    h = fmix32(((node * 0x9E3779B1) & M32) ^ ((d * 0x85EBCA77) & M32) ^ u)
    r = ((u + (h & 0xFFFF)) & M32) >> 16
    return float(np.uint32(r << 16).view(np.float32))


def drift(steps: int, inc_ulps: float, salted: bool, node: int = 12345, direction: int = 7):
    x = 1.0                         # bf16 ulp at 1.0 is 2^-7
    ulp = 2.0 ** -7
    for s in range(steps):
        d = direction | ((s << 5) if salted else 0)
        x = bf16_sr(x + inc_ulps * ulp, node, d)
    return (x - 1.0) / ulp


def test_step_term_keeps_a_sub_ulp_increment_unbiased():
    steps, inc = 4000, 0.3
    # with the step term the stored value advances by the increment on average
    got = np.mean([drift(steps, inc, True, node=n) for n in range(8)])
    assert abs(got - inc * steps) < 0.05 * inc * steps
    # without it, the first step that rounds down repeats the same pre-rounding value, hash and
    # rounding forever: the value freezes
    frozen = [drift(steps, inc, False, node=n) for n in range(8)]
    assert max(frozen) < 0.02 * inc * steps
