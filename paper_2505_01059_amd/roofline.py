"""Algorithmic work per rollout sample-step, counted from the rollout kernel's formulas.

One sample-step is one dynamics step plus its cost term for one candidate.
Counting rule: a fused multiply-add is 2 flops, an add / multiply / compare /
select 1; reciprocals and sin/cos are transcendentals, reported separately and
not included in the flop figure.  Terms that vanish structurally (the base
link's missing neighbour, the last link's missing successor) are not counted.

Chain without contact, n links, per evaluation of the accelerations (tension
solve and link accelerations):
    first row 25, interior rows 36 each, last row 20, back substitution 2(n-1)
    -> 38 n - 29 flops and n reciprocals.
Per RK4 step: 4 evaluations, joint-torque differences 2n - 1, stage updates
26 n, cost 6 n + 9  ->  186 n - 108 flops, 4 n reciprocals, 4 n sin/cos pairs.
Contact adds per mass and evaluation the position / velocity prefix sums (8),
the spring-damper and friction terms (about 10, plus one tanh) and the extra
right-hand-side and acceleration terms (6): 24 n flops per evaluation.
Point mass: Euler update 8, goal term 6, per obstacle 8, control term 5, sum 1.
"""


def flops_per_sample_step(dynamics: int, n_links: int = 0, n_obstacles: int = 0) -> int:
    if dynamics == 0:
        return 8 + 6 + 8 * n_obstacles + 5 + 1
    n = n_links
    base = 186 * n - 108
    if dynamics == 2:
        base += 4 * 24 * n
    return base


def transcendentals_per_sample_step(dynamics: int, n_links: int = 0) -> int:
    if dynamics == 0:
        return 0
    n = n_links
    t = 4 * n + 4 * n * 2           # reciprocals + sin and cos
    if dynamics == 2:
        t += 4 * n                  # tanh of the slip velocity
    return t


# MI355X (gfx950) peaks used for roofline fractions
PEAK_FP32_VECTOR_TFLOPS = 157.3     # 256 CUs x 2.4 GHz x 256 flop/clk/CU (packed FP32 issue)
PEAK_FP32_UNPACKED_TFLOPS = 78.6    # same chip issuing only unpacked FP32 FMA
PEAK_HBM_GBPS = 8000.0
