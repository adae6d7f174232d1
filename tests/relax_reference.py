"""Reference of the relaxation criterion for the tests: a plain host loop
over tdgl_energies_batch, against which the library's on-device test
(tdgl_relax) is compared.  "Relaxed at step n": the total energy changed by
less than rtol * max(|F(n)|, floor) over the last `check` steps."""
import numpy as np


def host_relax(ctx, floor, check=100, max_steps=20000, rtol=1e-6):
    """Step a batch context in calls of `check` until every instance has
    relaxed or max_steps.  Returns (relax step per instance, -1 if not
    relaxed; steps taken)."""
    f_prev = ctx.energies_batch()[0][:, 4].copy()
    done = np.full(len(f_prev), -1)
    steps = 0
    while steps < max_steps and (done < 0).any():
        ctx.step(check)
        steps += check
        f = ctx.energies_batch()[0][:, 4]
        ok = np.abs(f - f_prev) < rtol * np.maximum(np.abs(f), floor)
        done[(done < 0) & ok] = steps
        f_prev = f.copy()
    return done, steps
