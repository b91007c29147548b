"""High-wavenumber filter of a state (test infrastructure, see ``oracle/__init__``).

Sec. 4 proposes filtering high frequencies at the end of a time step to keep
Poisson ratios other than 1/4 stable, without fixing a filter. The filter
checked here is the definition the library documents, written out plainly:
every population becomes f - sigma (d4x f + d4y f) with the fourth difference
d4x g(x) = g(x-2) - 4 g(x-1) + 6 g(x) - 4 g(x+1) + g(x+2) (and the same along
y); an axis term is left out at a cell whose five-point stencil along that
axis would leave the grid through a non-periodic edge or cross the internal
rigid wall (between rows rigid_row - 1 and rigid_row)."""
import numpy as np

from workloads import BC_PERIODIC


def filter_state(p, f, sigma):
    """f: (9, ny, nx) FP64 state of problem p; returns the filtered copy."""
    f = np.asarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    px = p.bc[2] == BC_PERIODIC
    py = p.bc[0] == BC_PERIODIC
    rr = p.rigid_row
    out = f.copy()
    for y in range(ny):
        y_ok = (ny >= 5) if py else (2 <= y <= ny - 3)
        if rr > 0 and rr - 2 <= y <= rr + 1:
            y_ok = False
        for x in range(nx):
            x_ok = (nx >= 5) if px else (2 <= x <= nx - 3)
            for i in range(9):
                c = f[i, y, x]
                acc = 0.0
                if x_ok:
                    g = [f[i, y, (x + d) % nx] for d in (-2, -1, 1, 2)]
                    acc += g[0] - 4.0 * g[1] + 6.0 * c - 4.0 * g[2] + g[3]
                if y_ok:
                    g = [f[i, (y + d) % ny, x] for d in (-2, -1, 1, 2)]
                    acc += g[0] - 4.0 * g[1] + 6.0 * c - 4.0 * g[2] + g[3]
                out[i, y, x] = c - sigma * acc
    return out
