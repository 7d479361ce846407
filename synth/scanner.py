"""Cylindrical PET scanner geometry and span-1 sinogram LOR lists.

The projector interface of the paper takes a generic list of ray start and
end points (Sec. 2.2), so the scanner only exists to produce realistic LOR
endpoint lists.  Conventions:

* crystal ``c`` of ring ``r`` sits at
  ``(R cos(2 pi c / N), R sin(2 pi c / N), (r - (n_rings - 1) / 2) * pitch)``;
* sinogram view ``v`` in ``[0, N/2)`` and radial offset ``m`` in
  ``[-n_rad//2, n_rad - n_rad//2)`` map to the ordered crystal pair
  ``i = v + ((m mod 2) - m)/2 - N/4``, ``j = v + ((m mod 2) + m)/2 + N/4``
  (both mod N), so that ``j - i = N/2 + m`` and ``i + j = 2v + (m mod 2)``;
  the LOR's distance from the axis is ``R |sin(pi m / N)|``;
* planes are the ordered ring pairs ``(r1, r2)`` with ``|r1 - r2| <= max_rd``,
  ring ``r1`` major (span 1);
* the LOR of (m, v, plane) starts on crystal ``i`` of ring ``r1`` and ends on
  crystal ``j`` of ring ``r2``;
* storage order "RVP": radial slowest, then view, plane fastest -- the order
  the paper found fastest on its GPU (Sec. 3, Fig. 2 and 3 text).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch


def sinogram_planes(n_rings: int, max_rd: int) -> torch.Tensor:
    """Ordered ring pairs (r1, r2) with |r1 - r2| <= max_rd, r1 major. int64 [n_planes, 2]."""
    pairs = [(r1, r2) for r1 in range(n_rings) for r2 in range(n_rings) if abs(r1 - r2) <= max_rd]
    return torch.tensor(pairs, dtype=torch.int64)


def sinogram_crystal_pairs(n_crystals: int, n_rad: int, views=None):
    """Crystal indices (i, j) for every (radial, view) bin. Returns int64 tensors [n_rad, n_views]."""
    n = n_crystals
    if n % 4 != 0:
        raise ValueError("the sinogram mapping needs a crystal count divisible by 4")
    m = torch.arange(n_rad, dtype=torch.int64) - n_rad // 2
    v = torch.arange(n // 2, dtype=torch.int64) if views is None else torch.as_tensor(views, dtype=torch.int64)
    mm = m[:, None]
    par = torch.remainder(mm, 2)
    i = torch.remainder(v[None, :] + (par - mm) // 2 - n // 4, n)
    j = torch.remainder(v[None, :] + (par + mm) // 2 + n // 4, n)
    return i, j


@dataclass(frozen=True)
class CylinderScanner:
    radius: float  # mm
    n_rings: int
    ring_pitch: float  # mm
    n_crystals: int  # per ring

    def crystal_xyz(self, ring: torch.Tensor, crystal: torch.Tensor) -> torch.Tensor:
        """float64 [..., 3] centre of crystal ``crystal`` in ring ``ring``."""
        phi = (2.0 * math.pi / self.n_crystals) * crystal.to(torch.float64)
        z = (ring.to(torch.float64) - 0.5 * (self.n_rings - 1)) * self.ring_pitch
        return torch.stack([self.radius * torch.cos(phi), self.radius * torch.sin(phi), z], dim=-1)

    def crystal_table(self, device="cpu") -> torch.Tensor:
        """float32 [n_rings * n_crystals, 3]: row ring * n_crystals + crystal is that crystal's centre."""
        ring = torch.arange(self.n_rings).repeat_interleave(self.n_crystals)
        crystal = torch.arange(self.n_crystals).repeat(self.n_rings)
        return self.crystal_xyz(ring, crystal).to(torch.float32).contiguous().to(device)

    def sinogram_shape(self, n_rad: int, max_rd: int):
        return (n_rad, self.n_crystals // 2, int(sinogram_planes(self.n_rings, max_rd).shape[0]))

    def sinogram_lors(self, n_rad: int, max_rd: int, views=None, device="cpu", radial_chunk=None):
        """LOR endpoints of a span-1 sinogram in RVP order (plane fastest).

        Returns (xstart, xend), float32 contiguous [n_rad * n_views * n_planes, 3]
        on ``device``.  ``views`` restricts the sinogram to a subset of views
        (e.g. one OSEM subset); ``radial_chunk`` bounds temporary memory.
        """
        planes = sinogram_planes(self.n_rings, max_rd).to(device)
        ci, cj = sinogram_crystal_pairs(self.n_crystals, n_rad, views)
        ci, cj = ci.to(device), cj.to(device)
        n_views = ci.shape[1]
        n_planes = planes.shape[0]
        n = n_rad * n_views * n_planes
        xs = torch.empty((n, 3), dtype=torch.float32, device=device)
        xe = torch.empty((n, 3), dtype=torch.float32, device=device)
        step = radial_chunk or n_rad
        per_rad = n_views * n_planes
        for r0 in range(0, n_rad, step):
            r1 = min(n_rad, r0 + step)
            ii = ci[r0:r1, :, None].expand(r1 - r0, n_views, n_planes)
            jj = cj[r0:r1, :, None].expand(r1 - r0, n_views, n_planes)
            ra = planes[:, 0][None, None, :].expand_as(ii)
            rb = planes[:, 1][None, None, :].expand_as(ii)
            xs[r0 * per_rad : r1 * per_rad] = self.crystal_xyz(ra, ii).reshape(-1, 3).to(torch.float32)
            xe[r0 * per_rad : r1 * per_rad] = self.crystal_xyz(rb, jj).reshape(-1, 3).to(torch.float32)
        return xs, xe
