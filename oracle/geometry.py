"""Oracle geometry: the open-cavity MAC grid, its face classes and the control region.

TEST INFRASTRUCTURE ONLY (see the package header).

The flow domain follows the open-cavity configuration of Sec. 2 (Fig.
cavity_tikz, Table tabgeometry) in the simplified form used here: a channel
x in [0, L] x y in [0, 1] over a square cavity x in [x_cav, x_cav + 1] x
y in [-1, 0], lengths scaled by the cavity depth D = 1 (Re = U D / nu, Sec. 2).
Two test geometries reuse the same operators: a plain channel (no cavity, for
the plane Poiseuille pin) and a doubly periodic box [0, 2 pi]^2 (for the
Taylor-Green pins). The "paper" geometry takes the configuration of Sec. 2 and
the boundary conditions of Sec. 4.4 as far as they differ from the simplified
one: a channel of height H = 0.5 (Table tabgeometry) over the unit cavity, a
uniform inflow u = 1, a symmetry (slip) top wall, and a lower wall that is
no-slip only on L_1,slip = 0.4 upstream and L_2,slip = 0.75 downstream of the
cavity and slip beyond (Fig. cavity_tikz); the cavity walls are no-slip.

Layout (all arrays are numpy, y-row major, x fastest):
  cells   (NY, NX)      cell (i, j) centre ((i + 1/2) h, y0 + (j + 1/2) h)
  u faces (NY, NX + 1)  face (i, j) at x = i h between cells (i-1, j) and (i, j)
  v faces (NY + 1, NX)  face (i, j) at y = y0 + j h between cells (i, j-1) and (i, j)

Face classes: SOLID (no fluid cell on either side), ACTIVE (fluid on both
sides: carries a momentum equation), WALL (fluid on one side: no-slip, value
0), INFLOW (x = 0: prescribed parabola for u), OUTFLOW (x = L: convective).
"""
import numpy as np

SOLID, ACTIVE, WALL, INFLOW, OUTFLOW = 0, 1, 2, 3, 4

PAPER_HEIGHT = 0.5       # H of Table tabgeometry
PAPER_NOSLIP_UP = 0.4    # L_1,slip: no-slip lower wall for x_cav - 0.4 <= x <= x_cav
PAPER_NOSLIP_DOWN = 0.75  # L_2,slip: no-slip lower wall for x_cav + 1 <= x <= x_cav + 1.75


class Grid:
    """Uniform MAC grid of spacing h = 1/inv_h (2 pi / inv_h when periodic)."""

    def __init__(self, inv_h, geometry="cavity", x_cav=1.25, length=4.0):
        self.geometry = geometry
        self.inv_h = int(inv_h)
        n = self.inv_h
        if geometry == "periodic":
            self.h = 2.0 * np.pi / n
            self.NX, self.NY, self.y0 = n, n, 0.0
        elif geometry in ("cavity", "channel", "paper"):
            self.h = 1.0 / n
            self.NX = int(round(length * n))
            if abs(self.NX - length * n) > 1e-9:
                raise ValueError("channel length must be a multiple of h")
            if geometry in ("cavity", "paper"):
                height = 1.0 if geometry == "cavity" else PAPER_HEIGHT
                if (n * height) % 1 != 0:
                    raise ValueError("the channel height must be a multiple of h")
                self.NY, self.y0 = n + int(n * height), -1.0
                self.ic0 = int(round(x_cav * n))
                if abs(self.ic0 - x_cav * n) > 1e-9:
                    raise ValueError("cavity edge must lie on a grid line")
                self.ic1 = self.ic0 + n
            else:
                self.NY, self.y0 = n, 0.0
        else:
            raise ValueError(geometry)
        self.x_cav = x_cav
        self.length = length
        self.periodic = geometry == "periodic"
        h, NX, NY = self.h, self.NX, self.NY

        # cell centres and the fluid mask
        self.xc = (np.arange(NX) + 0.5) * h
        self.yc = self.y0 + (np.arange(NY) + 0.5) * h
        fluid = np.ones((NY, NX), dtype=bool)
        if geometry in ("cavity", "paper"):
            below = self.yc < 0.0
            inside = (np.arange(NX) >= self.ic0) & (np.arange(NX) < self.ic1)
            fluid[below, :] = False
            fluid[np.ix_(below, inside)] = True
        self.fluid = fluid

        # face classes
        def cell(j, i):
            if self.periodic:
                return True
            if i < 0 or i >= NX or j < 0 or j >= NY:
                return False
            return bool(fluid[j, i])

        ucls = np.zeros((NY, NX + 1), dtype=np.int8)
        for j in range(NY):
            for i in range(NX + 1):
                if self.periodic:
                    ucls[j, i] = ACTIVE if i < NX else SOLID  # i = NX duplicates i = 0
                    continue
                w, e = cell(j, i - 1), cell(j, i)
                if i == 0:
                    ucls[j, i] = INFLOW if e else SOLID
                elif i == NX:
                    ucls[j, i] = OUTFLOW if w else SOLID
                elif w and e:
                    ucls[j, i] = ACTIVE
                elif w or e:
                    ucls[j, i] = WALL
        vcls = np.zeros((NY + 1, NX), dtype=np.int8)
        for j in range(NY + 1):
            for i in range(NX):
                if self.periodic:
                    vcls[j, i] = ACTIVE if j < NY else SOLID
                    continue
                s, nn = cell(j - 1, i), cell(j, i)
                if s and nn:
                    vcls[j, i] = ACTIVE
                elif s or nn:
                    vcls[j, i] = WALL
        self.ucls, self.vcls = ucls, vcls
        self.ncells = int(fluid.sum())

        # sign of the mirrored u value across a wall parallel to x (the u face beyond is SOLID or
        # outside the box): -1 no-slip (u = 0 half a cell away), +1 slip (du/dy = 0)
        self.mirror_S = -np.ones((NY, NX + 1))
        self.mirror_N = -np.ones((NY, NX + 1))
        self.inflow = "parabola"
        self.u_convective = 2.0 / 3.0  # bulk speed of the parabola 4 y (1 - y)
        if geometry == "paper":
            self.inflow = "uniform"
            self.u_convective = 1.0
            self.mirror_N[NY - 1, :] = 1.0  # symmetry top
            jc = n  # first channel row
            xs0, xs1 = x_cav - PAPER_NOSLIP_UP, x_cav + 1.0 + PAPER_NOSLIP_DOWN
            for i in range(NX + 1):
                x = i * h
                if (x < xs0 or x > xs1) and ucls[jc - 1, i] == SOLID:
                    self.mirror_S[jc, i] = 1.0

    # ------------------------------------------------------------------ inflow
    def inflow_profile(self):
        """Inflow on the x = 0 faces: the parabola u = 4 y (1 - y) (unit centreline speed), or
        u = 1 (the paper geometry's uniform inflow, Sec. 4.4)."""
        y = self.yc
        prof = np.ones_like(y) if self.inflow == "uniform" else 4.0 * y * (1.0 - y)
        return np.where(self.ucls[:, 0] == INFLOW, prof, 0.0)


def control_cells(grid, region="column", box=None):
    """Row-major list of the control cells (j, i) of a forcing region.

    'column' : the cavity plus the channel column above it, x in [x_cav, x_cav+1]
               and every y, 2/h^2 cells. This reading makes the three control
               sizes quoted for the workloads (2048 per component at h = 1/32,
               32768 per component at h = 1/128, 65536 in total) agree.
    'cavity' : the cavity cells only, 1/h^2 cells.
    'box'    : fluid cells whose centre lies in [x0, x1] x [y0, y1] (the
               paper's actuation window of Sec. 4.1 is such a box).
    """
    cells = []
    for j in range(grid.NY):
        for i in range(grid.NX):
            if not grid.fluid[j, i]:
                continue
            x, y = grid.xc[i], grid.yc[j]
            if region == "column":
                ok = grid.x_cav < x < grid.x_cav + 1.0
            elif region == "cavity":
                ok = grid.x_cav < x < grid.x_cav + 1.0 and y < 0.0
            elif region == "box":
                x0, x1, y0, y1 = box
                ok = x0 <= x <= x1 and y0 <= y <= y1
            else:
                raise ValueError(region)
            if ok:
                cells.append((j, i))
    return cells
