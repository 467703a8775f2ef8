"""Measurements on result fields shared by the oracle pins and the GPU tests
(no product code, no oracle arithmetic)."""

def front_radius(prof):
    """Outermost local maximum of significant height of a radial profile,
    refined by a parabola through its neighbours (the position of a pulse
    front; the decaying diffusive hump left at the centre can be higher)."""
    big = prof > 0.05 * prof.max()
    peaks = [r for r in range(1, prof.size - 1)
             if big[r] and prof[r] >= prof[r - 1] and prof[r] > prof[r + 1]]
    r = peaks[-1]
    a, b, c = prof[r - 1], prof[r], prof[r + 1]
    return r + 0.5 * (a - c) / (a - 2 * b + c)
