"""Listmode TOF OSEM on the fused, batched kernels of libppmi.so.

The paper runs listmode OSEM with all operations on the GPU (Sec. 2.6); here
one subset update of any number of frames sharing an image grid is two
kernel launches (pp_lm_osem_subset_batched, pp_osem_update_batched) driven by a slot
table in device memory, so a sequence of steps can be captured once into a
HIP graph and replayed for any mix of frames.

Reading of the method used throughout (same as the FP64 oracle): subset j
holds the events with index e mod n_sub == j in the frame's own event order;
x0 = 1 where the sensitivity is positive, else 0; each subset update is
x <- x * A_j^T (1 / (A_j x + bg)) / (sens / n_sub), zero where sens == 0.
With the image-based resolution model (the paper's reconstructions use a 3D
Gaussian of 4.5 mm FWHM, Sec. 2.6) the system model is A G: the forward
projects G x, the back projection is followed by G, and sens = G A^T 1.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import COsemSlot, as_geom, as_tof, check, load, ptr, stream_of
from .projectors import back, fwhm3, gather_crystal_events, gather_events, pp_gauss3d, presort, presort_crystals

SLOT_BYTES = ctypes.sizeof(COsemSlot)
RES_FWHM_MM = 4.5  # the paper's resolution model


def prepare_frame(xstart, xend, tof_bin, geom, tof, n_sub):
    """Device copies of a frame's events in subset-major order, presorted inside each subset."""
    order = presort(xstart, xend, geom, tof_bin, tof, n_sub=n_sub)
    return gather_events(xstart, xend, tof_bin, order)


def prepare_crystal_frame(crystal_xyz, pair, tof_bin, geom, tof, n_sub):
    """prepare_frame for crystal-index events: (pair, tof_bin) in subset-major, presorted order."""
    order = presort_crystals(crystal_xyz, pair, geom, tof_bin, tof, n_sub=n_sub)
    return gather_crystal_events(pair, tof_bin, order)


def sensitivity(lor_start, lor_end, geom, chunk=1 << 26, res_fwhm=None):
    """Non-TOF back projection of ones over a LOR set (the scanner's sinogram LORs), followed by
    the resolution model when `res_fwhm` is given."""
    g = as_geom(geom)
    dev = lor_start.device
    sens = torch.zeros(g.dim, dtype=torch.float32, device=dev)
    for a in range(0, lor_start.shape[0], chunk):
        b = min(lor_start.shape[0], a + chunk)
        ones = torch.ones(b - a, dtype=torch.float32, device=dev)
        back(lor_start[a:b], lor_end[a:b], g, ones, img=sens)
    if res_fwhm is not None:
        out, tmp = torch.empty_like(sens), torch.empty_like(sens)
        pp_gauss3d(sens, out, tmp, g, res_fwhm)
        sens = out
    return sens


class SlotTable:
    """Host mirror + device copy of a pp_frame_desc_t array for one image grid."""

    def __init__(self, capacity, device):
        self.capacity = int(capacity)
        self.host = (COsemSlot * self.capacity)()
        self.pinned = torch.empty(self.capacity * SLOT_BYTES, dtype=torch.uint8, pin_memory=True)
        self.dev = torch.zeros(self.capacity * SLOT_BYTES, dtype=torch.uint8, device=device)
        self._copied = None

    def set(self, i, xs, xe, tb, x, acc, sens, n_sub, steps, bg, x_fwd=None, tmp=None, n_events=None):
        """Slot i <- a frame.  x_fwd and tmp (both or neither): the resolution model's G x (set
        before the first step) and its scratch image."""
        if (x_fwd is None) != (tmp is None):
            raise ValueError("x_fwd and tmp go together")
        if not 0 <= int(i) < self.capacity:
            raise IndexError(f"slot {i} outside the table of {self.capacity}")
        n_ev = xs.shape[0] if n_events is None else int(n_events)
        if int(n_sub) < 1 or n_ev < 0 or int(steps) < 0:
            raise ValueError("a slot needs n_sub >= 1, n_events >= 0 and steps >= 0")
        self.clear(i)
        s = self.host[i]
        s.xstart = None if xs is None else xs.data_ptr()
        s.xend = None if xe is None else xe.data_ptr()
        s.tof_bin = tb.data_ptr()
        s.x, s.acc, s.sens = x.data_ptr(), acc.data_ptr(), sens.data_ptr()
        s.x_fwd = None if x_fwd is None else x_fwd.data_ptr()
        s.tmp = None if tmp is None else tmp.data_ptr()
        s.n_events = n_ev
        s.bg = float(bg)
        s.n_sub = int(n_sub)
        s.subset = 0
        s.steps_left = int(steps)
        s.active = 1

    def set_crystals(self, i, crystal_xyz, pair, tb, x, acc, sens, n_sub, steps, bg, x_fwd=None, tmp=None):
        """Slot i <- a frame of crystal-index events (pair [n, 2] int32 into crystal_xyz)."""
        if pair.dtype != torch.int32 or pair.dim() != 2 or pair.shape[1] != 2 or pair.data_ptr() % 8:
            raise ValueError("pair must be 8-byte aligned int32 [n, 2]")
        if crystal_xyz.dtype != torch.float32 or crystal_xyz.dim() != 2 or crystal_xyz.shape[1] != 3:
            raise ValueError("crystal_xyz must be float32 [n_crystals, 3]")
        self.set(i, None, None, tb, x, acc, sens, n_sub, steps, bg, x_fwd, tmp, n_events=pair.shape[0])
        s = self.host[i]
        s.crystal_pair, s.crystal_xyz, s.n_crystals = pair.data_ptr(), crystal_xyz.data_ptr(), crystal_xyz.shape[0]

    def clear(self, i):
        ctypes.memset(ctypes.addressof(self.host[i]), 0, SLOT_BYTES)

    def upload(self):
        """Recompute chunk offsets and copy the table to the device (stream-ordered)."""
        lib = load()
        acc = 0
        for s in self.host:
            s.chunk_begin = acc
            if s.active:
                acc += int(lib.pp_osem_chunks(s.n_events, s.n_sub))
        if self._copied is not None:
            self._copied.synchronize()  # the previous copy has read the pinned buffer
        ctypes.memmove(self.pinned.data_ptr(), ctypes.addressof(self.host), self.capacity * SLOT_BYTES)
        self.dev.copy_(self.pinned, non_blocking=True)
        self._copied = torch.cuda.Event()
        self._copied.record()

    def advance_host(self, steps):
        """Mirror what `steps` device steps do to live slots (subset, steps_left)."""
        for s in self.host:
            for _ in range(steps):
                if s.active and s.steps_left > 0:
                    s.subset = (s.subset + 1) % s.n_sub
                    s.steps_left -= 1


def osem_steps(table: SlotTable, geom, tof, n_steps=1, res_fwhm=None):
    """Enqueue n_steps subset updates for every live slot of the table (current stream);
    res_fwhm (mm) is the resolution model of the slots that have x_fwd set."""
    g, t = as_geom(geom), as_tof(tof)
    lib = load()
    if t.per_ray:
        raise ValueError("listmode OSEM takes one TOF kernel for every event (no per-ray parameters)")
    gc, tc = g.c(), t.c()
    fw = None if res_fwhm is None else fwhm3(res_fwhm)
    st = stream_of(table.dev)
    for _ in range(n_steps):
        check(lib.pp_lm_osem_subset_batched(ptr(table.dev), table.capacity, gc, tc, st))
        check(lib.pp_osem_update_batched(ptr(table.dev), table.capacity, gc, fw, st))


def capture_steps(table: SlotTable, geom, tof, n_steps=1, res_fwhm=None):
    """A HIP graph of n_steps subset updates over the table (replay serves any slot mix)."""
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream(device=table.dev.device)
    cap.wait_stream(torch.cuda.current_stream(table.dev.device))
    with torch.cuda.graph(graph, stream=cap):
        osem_steps(table, geom, tof, n_steps, res_fwhm)
    torch.cuda.current_stream(table.dev.device).wait_stream(cap)
    return graph


def init_image(sens):
    x = torch.empty_like(sens)
    check(load().pp_osem_init(ptr(x), ptr(sens), sens.numel(), stream_of(x)))
    return x


def res_buffers(x, geom, res_fwhm):
    """(x_fwd = G x, tmp) for a frame that uses the resolution model."""
    x_fwd, tmp = torch.empty_like(x), torch.empty_like(x)
    pp_gauss3d(x, x_fwd, tmp, geom, res_fwhm)
    return x_fwd, tmp


def lm_osem_crystals(crystal_xyz, pair, tof_bin, geom, tof, sens, n_iter, n_sub, bg=0.1, x0=None, res_fwhm=None):
    """lm_osem for crystal-index events (pair [n, 2] int32 into crystal_xyz [n_crystals, 3])."""
    g = as_geom(geom)
    pr, tb = prepare_crystal_frame(crystal_xyz, pair, tof_bin, g, tof, n_sub)
    x = init_image(sens) if x0 is None else x0.clone()
    acc = torch.zeros_like(sens)
    x_fwd = tmp = None
    if res_fwhm is not None:
        x_fwd, tmp = res_buffers(x, g, res_fwhm)
    table = SlotTable(1, pair.device)
    table.set_crystals(0, crystal_xyz, pr, tb, x, acc, sens, n_sub, n_iter * n_sub, bg, x_fwd, tmp)
    table.upload()
    osem_steps(table, g, tof, n_iter * n_sub, res_fwhm)
    torch.cuda.current_stream(x.device).synchronize()
    del pr, tb
    return x


def lm_osem(xstart, xend, tof_bin, geom, tof, sens, n_iter, n_sub, bg=0.1, x0=None, res_fwhm=None):
    """Listmode TOF OSEM of one frame (events in the frame's own order) on the fused kernels;
    with `res_fwhm` (mm) the system model includes the Gaussian resolution model (then `sens`
    must include it too, see `sensitivity`)."""
    g = as_geom(geom)
    xs, xe, tb = prepare_frame(xstart, xend, tof_bin, g, tof, n_sub)
    x = init_image(sens) if x0 is None else x0.clone()
    acc = torch.zeros_like(sens)
    x_fwd = tmp = None
    if res_fwhm is not None:
        x_fwd, tmp = res_buffers(x, g, res_fwhm)
    table = SlotTable(1, xstart.device)
    table.set(0, xs, xe, tb, x, acc, sens, n_sub, n_iter * n_sub, bg, x_fwd, tmp)
    table.upload()
    osem_steps(table, g, tof, n_iter * n_sub, res_fwhm)
    torch.cuda.current_stream(x.device).synchronize()
    del xs, xe, tb
    return x
