"""The paper's weight-iteration schedule (Sec. 3: Eq. 6, Eq. 7 and the
thermalisation rule) driving the oracle chain -- TEST INFRASTRUCTURE.

Per iteration, with W walkers on an L x L lattice (N = L^2 spins, N+1 energy
bins):
  * w = max(w', 10), w' the width in bins of the energy range the previous
    iteration's histogram covered (lowest to highest visited bin; 0 before
    the first iteration), so that the full range is w = N + 1;
  * N_therm = f_therm * w unrecorded attempts per walker (f_therm = 30);
  * N_updates = floor(x) + 1 recorded attempts per walker, where
    x = 6 w^z / W (z = 2.25, Eq. 7) up to and including the first iteration
    whose w is the full range, and x grows by the factor 1.1 in every
    iteration after that;
  * the weights are updated by Eq. 4; from the first iteration whose w is
    the full range on, the run stops after the first iteration whose
    Kullback-Leibler divergence d_k (Eq. 6, P = H / sum H, Q uniform over
    the reachable bins of the previous iteration's range) is below 10^-4 --
    or, with the alternative rule of App. A, whose Chebyshev distance
    d_c = max |H / m - 1| over the reachable bins (m = sum H / their number)
    is below 0.05.
Readings where the text leaves room: the growth phase, once entered, is kept
even if a later iteration covers a narrower range; the stop test waits for
the full range, because before it Q need not cover the current histogram
and d_k can come out negative, which would end the run at once.
"""
import math


def run_paper_schedule(o, z=2.25, f_therm=30, growth=1.1, dk_flat=1e-4, w_min=10,
                       max_iterations=1000, stop="kl", dc_flat=0.05):
    """Iterate the oracle instance ``o`` (an ``OracleMuca``) by the schedule,
    stopping on d_k < dk_flat (stop="kl") or d_c < dc_flat
    (stop="chebyshev").  Returns (converged, steps) with one dict per
    iteration."""
    assert stop in ("kl", "chebyshev")
    x = None
    full = False
    steps = []
    for _ in range(max_iterations):
        w = max(o.width_prev, w_min)
        if full:
            x = x * growth
        else:
            x = 6.0 * w ** z / o.W
            full = w == o.N + 1
        n_updates = int(math.floor(x)) + 1
        n_therm = f_therm * w
        info = o.iterate_attempts(n_therm, n_updates)
        steps.append({"therm_attempts": n_therm, "update_attempts": n_updates, "width": w,
                      "covered": info["width"], "kl_divergence": info["kl_divergence"],
                      "chebyshev": info["chebyshev"], "flatness": info["flatness"]})
        d, below = (info["chebyshev"], dc_flat) if stop == "chebyshev" else (info["kl_divergence"], dk_flat)
        if full and d < below:
            return True, steps
    return False, steps
