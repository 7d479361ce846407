"""Image grids and seeded voxel phantoms.

Image convention (shared by every part of the repository): a float array in
C order ``[dim0][dim1][dim2]`` (axis 2 fastest in memory); voxel ``(i, j, k)``
has its *centre* at ``origin + (i * vs0, j * vs1, k * vs2)`` in mm.  A centred
grid has ``origin = -(dim - 1) / 2 * voxsize``.  Phantoms are voxelised by
evaluating the analytic object at voxel centres.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch


@dataclass(frozen=True)
class ImageGrid:
    dim: tuple  # (n0, n1, n2)
    voxsize: tuple  # mm
    origin: tuple = field(default=None)  # centre of voxel (0,0,0), mm

    def __post_init__(self):
        if self.origin is None:
            object.__setattr__(
                self, "origin", tuple(-(n - 1) / 2.0 * h for n, h in zip(self.dim, self.voxsize))
            )

    @property
    def n_vox(self) -> int:
        return int(self.dim[0]) * int(self.dim[1]) * int(self.dim[2])

    def centres(self, device="cpu"):
        """Voxel-centre coordinates as three float64 tensors broadcastable to ``dim``."""
        axes = []
        for a in range(3):
            c = self.origin[a] + self.voxsize[a] * torch.arange(self.dim[a], dtype=torch.float64, device=device)
            shape = [1, 1, 1]
            shape[a] = self.dim[a]
            axes.append(c.reshape(shape))
        return axes

    def shifted(self, dx):
        return ImageGrid(self.dim, self.voxsize, tuple(o + d for o, d in zip(self.origin, dx)))


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def cylinder_sphere_phantom(grid: ImageGrid, seed: int, cyl_radius=100.0, n_spheres=3,
                            sphere_radius=(8.0, 15.0), sphere_value=4.0, device="cpu"):
    """Uniform cylinder (value 1, full axial extent) with hot spheres painted on top.

    Sphere radii are U(sphere_radius); centres are drawn uniformly in the
    cylinder (transaxially inside ``cyl_radius - r``, axially inside the grid).
    Returns float32 ``dim``.
    """
    g = _gen(seed)
    x, y, z = grid.centres(device)
    img = ((x * x + y * y) <= cyl_radius**2).to(torch.float64).expand(*grid.dim).clone()
    zext = 0.5 * (grid.dim[2] - 1) * grid.voxsize[2]
    for _ in range(n_spheres):
        r = sphere_radius[0] + (sphere_radius[1] - sphere_radius[0]) * torch.rand((), generator=g, dtype=torch.float64).item()
        rho = (cyl_radius - r) * torch.sqrt(torch.rand((), generator=g, dtype=torch.float64)).item()
        ang = 2.0 * torch.pi * torch.rand((), generator=g, dtype=torch.float64).item()
        cz = grid.origin[2] + zext + (2.0 * torch.rand((), generator=g, dtype=torch.float64).item() - 1.0) * zext
        cx, cy = rho * float(torch.cos(torch.tensor(ang))), rho * float(torch.sin(torch.tensor(ang)))
        inside = ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) <= r * r
        img[inside.expand(*grid.dim)] = sphere_value
    return img.to(torch.float32).contiguous()


def ellipsoid_lesion_phantom(grid: ImageGrid, seed: int, semi_axes=(150.0, 110.0, 60.0), n_lesions=10,
                             lesion_radius=(5.0, 20.0), value_range=(0.0, 8.0), centre=(0.0, 0.0, 0.0),
                             device="cpu"):
    """Ellipsoid of value 1 with ``n_lesions`` spheres painted in order.

    Lesion radii are U(lesion_radius), values U(value_range), centres drawn
    uniformly inside the ellipsoid shrunk by the radius.  ``centre`` shifts
    the whole object (used as a rigid-motion stand-in).  Returns float32 ``dim``.
    """
    g = _gen(seed)
    x, y, z = grid.centres(device)
    x, y, z = x - centre[0], y - centre[1], z - centre[2]
    a, b, c = semi_axes
    img = ((x / a) ** 2 + (y / b) ** 2 + (z / c) ** 2 <= 1.0).to(torch.float64).expand(*grid.dim).clone()
    for _ in range(n_lesions):
        u = torch.rand(6, generator=g, dtype=torch.float64)
        r = lesion_radius[0] + (lesion_radius[1] - lesion_radius[0]) * u[0].item()
        val = value_range[0] + (value_range[1] - value_range[0]) * u[1].item()
        # uniform point in the unit ball, scaled to the shrunken ellipsoid
        direc = torch.randn(3, generator=g, dtype=torch.float64)
        direc = direc / direc.norm()
        rad = u[2].item() ** (1.0 / 3.0)
        cx = direc[0].item() * rad * max(a - r, 1.0)
        cy = direc[1].item() * rad * max(b - r, 1.0)
        cz = direc[2].item() * rad * max(c - r, 1.0)
        inside = ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) <= r * r
        img[inside.expand(*grid.dim)] = val
    return img.to(torch.float32).contiguous()
