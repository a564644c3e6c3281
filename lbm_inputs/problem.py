"""Problem description handed unchanged to the GPU library and the oracle."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

#: one cut link: fluid node (x, y), direction dir (1..8) pointing into the
#: solid, wall fraction q in (0, 1] (Eq. 6), wall velocity at the cut point.
LINK_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("dir", "<i4"),
                       ("pad", "<i4"), ("q", "<f8"), ("uwx", "<f8"),
                       ("uwy", "<f8")])

RULES = ("halfway", "fh", "mls", "ibb_linear", "ibb_quadratic", "zhao_yong")
FIXES = ("none", "A", "B", "bao")
EOSES = ("none", "exp", "cs")
COLLISIONS = ("bgk", "mrt")


@dataclass
class Problem:
    """A D2Q9 domain with solid obstacles, periodic in y and, unless
    ``open_x`` is set (velocity inlet at x = 0, outflow at x = nx - 1),
    in x.

    Arrays are indexed [y, x].  ``rho_wall`` is the constant virtual wall
    density of the contact-angle treatment; it is read at solid nodes only.
    """

    nx: int
    ny: int
    solid: np.ndarray            # uint8 (ny, nx), 1 = solid
    links: np.ndarray            # LINK_DTYPE (nlinks,)
    rho0: np.ndarray             # float64 (ny, nx), initial density
    rho_wall: np.ndarray         # float64 (ny, nx), read at solid nodes
    eos: str = "none"
    eos_params: tuple = (0.0, 0.0, 0.0, 0.0)   # exp: psi0, rho0; cs: a, b, R, T
    G: float = 0.0
    gravity: tuple = (0.0, 0.0)
    collision: str = "bgk"
    tau: float = 1.0
    mrt_s: tuple = (1.0,) * 9
    rule: str = "halfway"
    fix: str = "none"
    ux0: Optional[np.ndarray] = None
    uy0: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)
    open_x: bool = False         # velocity inlet at x = 0, outlet at nx - 1
    inlet_u: float = 0.0         # inlet velocity (x component)

    def __post_init__(self):
        assert self.rule in RULES, self.rule
        assert self.fix in FIXES, self.fix
        assert self.eos in EOSES, self.eos
        assert self.collision in COLLISIONS, self.collision
        self.solid = np.ascontiguousarray(self.solid, dtype=np.uint8)
        self.rho0 = np.ascontiguousarray(self.rho0, dtype=np.float64)
        self.rho_wall = np.ascontiguousarray(self.rho_wall, dtype=np.float64)
        self.links = np.ascontiguousarray(self.links, dtype=LINK_DTYPE)
        assert self.solid.shape == (self.ny, self.nx)
        assert self.rho0.shape == (self.ny, self.nx)
        assert self.rho_wall.shape == (self.ny, self.nx)
        for v in (self.ux0, self.uy0):
            assert v is None or v.shape == (self.ny, self.nx)

    def with_(self, **kw) -> "Problem":
        """Copy with some fields replaced."""
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)

    @property
    def fluid_nodes(self) -> int:
        return int(self.nx * self.ny - int(self.solid.sum()))
