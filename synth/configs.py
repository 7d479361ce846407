"""The five synthetic workloads (scanner, sinogram, image grid, phantom, TOF, events).

Sizes follow the workload definitions this repository is measured on; the
paper's own GE Discovery MI / NEMA workloads (Sec. 2.6) are replaced by these
seeded stand-ins.  Every random draw takes an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass

from .phantom import ImageGrid, cylinder_sphere_phantom, ellipsoid_lesion_phantom
from .scanner import CylinderScanner

FWHM_TO_SIGMA = 1.0 / 2.355


@dataclass(frozen=True)
class TofSpec:
    bin_width: float  # mm
    sigma: float  # mm
    n_sigmas: float
    n_bins: int
    center_offset: float = 0.0


@dataclass(frozen=True)
class SinoSpec:
    scanner: CylinderScanner
    n_rad: int
    max_rd: int

    @property
    def shape(self):
        return self.scanner.sinogram_shape(self.n_rad, self.max_rd)

    @property
    def n_lors(self):
        a, b, c = self.shape
        return a * b * c

    def lors(self, views=None, device="cpu", radial_chunk=None):
        return self.scanner.sinogram_lors(self.n_rad, self.max_rd, views=views, device=device,
                                          radial_chunk=radial_chunk)


# --- small plain case: 64 views x 63 radial x 16 ring pairs = 64,512 LORs ---------
SCANNER_SMALL = CylinderScanner(radius=200.0, n_rings=4, ring_pitch=4.0, n_crystals=128)
SINO_SMALL = SinoSpec(SCANNER_SMALL, n_rad=63, max_rd=3)
GRID_SMALL = ImageGrid((64, 64, 8), (4.0, 4.0, 2.0))


def phantom_small(device="cpu"):
    return cylinder_sphere_phantom(GRID_SMALL, seed=1, cyl_radius=100.0, n_spheres=3,
                                   sphere_radius=(8.0, 15.0), sphere_value=4.0, device=device)


SEED_SMALL_Y = 2

# --- clinical size: 400 radial x 380 views x 2,204 planes = 335,008,000 LORs --------
SCANNER_CLIN = CylinderScanner(radius=410.0, n_rings=64, ring_pitch=4.0, n_crystals=760)
SINO_CLIN = SinoSpec(SCANNER_CLIN, n_rad=400, max_rd=20)
GRID_CLIN = ImageGrid((215, 215, 71), (1.65, 1.65, 2.0))


def phantom_clin(device="cpu", centre=(0.0, 0.0, 0.0), grid=GRID_CLIN, seed=3):
    return ellipsoid_lesion_phantom(grid, seed=seed, semi_axes=(150.0, 110.0, 60.0), n_lesions=10,
                                    lesion_radius=(5.0, 20.0), value_range=(0.0, 8.0),
                                    centre=centre, device=device)


SEED_CLIN_Y = 4

# --- TOF: 29 bins of 28 mm, FWHM 58.5 mm, truncated at 3 sigma ----------------------
TOF_CLIN = TofSpec(bin_width=28.0, sigma=58.5 * FWHM_TO_SIGMA, n_sigmas=3.0, n_bins=29)
SEED_TOF_Y = 5

# --- TOF listmode: 40M events from the clinical phantom ----------------------------
N_EVENTS_LM = 40_000_000
SEED_EVENTS = 6
GRID_DL = ImageGrid((128, 128, 64), (2.78, 2.78, 2.78))  # batch-of-8 autograd images
SEEDS_DL_IMAGES = tuple(range(7, 15))
SEED_FD_VOXELS = 15
BG_DL = 0.1

# --- serving: 256 short-frame TOF LM-OSEM requests ---------------------------------
N_REQUESTS = 256
SEED_SERVE = 16
SERVE_EVENTS_RANGE = (500_000, 20_000_000)  # log-uniform
SERVE_GRIDS = (GRID_DL, GRID_CLIN)
OSEM_ITERS = 3
OSEM_SUBSETS = 8
OSEM_BG = 0.1
