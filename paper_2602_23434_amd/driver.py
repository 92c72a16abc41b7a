"""Device-memory plumbing around the C ABI.

A :class:`Run` takes a workload from :mod:`paper_2602_23434_amd.inputs`,
allocates its fields, particles (both buffer sets) and moment grids as torch
tensors on the GPU, describes them to libpl.so as ``pl_item`` records, and
forwards step / sort / pack / unpack calls.  torch supplies memory and the
stream only; every step of the particle update runs in libpl.so's kernels.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import binding as B

KIND = {"lorentz": B.PL_LORENTZ, "dust": B.PL_DUST, "tracer": B.PL_TRACER}
SHAPE = {"cic": B.PL_CIC, "tsc": B.PL_TSC}
CH_NAMES = ["rho", "J0", "J1", "J2", "F0", "F1", "F2", "eng"]


def _ptr(t):
    return t.data_ptr() if t is not None else None


class Run:
    """One context plus the device arrays of every item of a workload."""

    def __init__(self, wl, prec=B.PL_F64, algo=B.PL_ALGO_PLAIN, key_mode=None, block=0,
                 tile=None, c=1.0, weights=True, ids=True, fp=False, eng=True, sort_buffers=True,
                 tune_cache=None, channels=None, device="cuda", spectra=False, spectra_sets=2, capacity=None):
        import torch

        self.torch = torch
        self.wl = wl
        if key_mode is None:
            key_mode = B.PL_KEY_TILE_RUN if algo == B.PL_ALGO_RUNS else B.PL_KEY_TILE
        self.prec = prec
        self.algo = algo
        self.dev = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.dev)
        self.ndim = wl.boxes[0].ndim
        fdt = torch.float64 if prec == B.PL_F64 else torch.float32
        self.fdt = fdt

        nb = len(wl.boxes)
        self._boxes = (B.pl_box_desc * nb)()
        for i, bx in enumerate(wl.boxes):
            for a in range(3):
                self._boxes[i].n[a] = bx.n[a]
                self._boxes[i].dx[a] = bx.dx[a]
                self._boxes[i].tile[a] = tile[a] if tile else 0
        ns = len(wl.species)
        self._species = (B.pl_species_desc * ns)()
        for i, sp in enumerate(wl.species):
            self._species[i].kind = KIND[sp.kind]
            self._species[i].q = sp.q
            self._species[i].m = sp.m
            self._species[i].weight = sp.weight
            self._species[i].t_stop = sp.t_stop
            self._species[i].rk_stages = getattr(sp, "rk_stages", 2)
        d = B.pl_init_desc()
        d.ndim = self.ndim
        d.prec = prec
        d.shape = SHAPE[wl.shape]
        d.algo = algo
        d.key_mode = key_mode
        d.c = c
        d.nboxes = nb
        d.boxes = self._boxes
        d.nspecies = ns
        d.species = self._species
        d.max_items = len(wl.items)
        self.capacity = [max(it.particles.n, capacity or 0) for it in wl.items]
        d.max_np = max(1, max(self.capacity))
        d.block = block
        d.stream = self.stream.cuda_stream
        d.tune_cache = tune_cache.encode() if tune_cache else None
        self.desc = d
        self.ctx = B.pl_part_init(d)

        with torch.cuda.stream(self.stream):
            self.fields = []
            for bx in wl.boxes:
                self.fields.append({k: torch.from_numpy(v).to(self.dev) for k, v in bx.fields.items()})
            self.items = (B.pl_item * len(wl.items))()
            self.parts = []
            self.moms = []
            self.mom_blocks = []
            for i, it in enumerate(wl.items):
                bx = wl.boxes[it.box]
                sp = wl.species[it.species]
                kind = KIND[sp.kind]
                n = self.capacity[i]
                sets = []
                for s in range(2 if sort_buffers else 1):
                    st = {
                        "x": [torch.empty(n, dtype=fdt, device=self.dev) for _ in range(self.ndim)],
                        "u": [torch.empty(n, dtype=fdt, device=self.dev) for _ in range(3)],
                        "cell": torch.empty(n, dtype=torch.int32, device=self.dev) if prec == B.PL_F32_OFFSET else None,
                        "w": torch.empty(n, dtype=fdt, device=self.dev) if weights else None,
                        "id": torch.empty(n, dtype=torch.int64, device=self.dev) if ids else None,
                    }
                    sets.append(st)
                ntiles = 1
                tl = [self._boxes[it.box].tile[a] or 0 for a in range(3)]
                extra = {
                    "fp": [torch.zeros(n, dtype=fdt, device=self.dev) for _ in range(3)] if fp else None,
                    "tile_start": torch.zeros(bx.n[0] * bx.n[1] * bx.n[2] + 1, dtype=torch.int32, device=self.dev),
                    # run table sized for one tile per cell (the most tiles a box can have)
                    "runs": (torch.zeros(B.runs_len(n, bx.n[0] * bx.n[1] * bx.n[2]), dtype=torch.int32, device=self.dev)
                             if algo == B.PL_ALGO_RUNS else None),
                    "eng": None, "chi": None,
                }
                if spectra:
                    # every particle starts with the workload's template spectrum
                    e0 = torch.from_numpy(np.ascontiguousarray(wl.notes["eng0"])).to(self.dev)
                    c0 = torch.from_numpy(np.ascontiguousarray(wl.notes["chi0"])).to(self.dev)
                    nbins = e0.shape[0]
                    extra["eng"] = [torch.empty((n, nbins), dtype=torch.float64, device=self.dev)
                                    for _ in range(spectra_sets)]
                    extra["chi"] = [torch.empty((n, nbins), dtype=torch.float64, device=self.dev)
                                    for _ in range(spectra_sets)]
                    extra["eng"][0].copy_(e0.expand(n, nbins))
                    extra["chi"][0].copy_(c0.expand(n, nbins))
                self.parts.append({"sets": sets, **extra})
                shape = (bx.n[2], bx.n[1], bx.n[0])
                # every channel of the item is a view of one block, so zeroing the
                # moments is a single fill
                want = set(channels) if channels is not None else set(CH_NAMES)
                if kind == B.PL_LORENTZ:
                    nch = ("rho" in want) + 3 * ("J0" in want) + 3 * ("F0" in want) + (bool(eng) and "eng" in want)
                elif kind == B.PL_DUST:
                    nch = ("rho" in want) + 3 * ("F0" in want)
                else:
                    nch = 0
                block = torch.zeros((nch,) + shape, dtype=torch.float64, device=self.dev)
                used = iter(range(nch))
                z = lambda: block[next(used)]
                mo = {}
                if kind == B.PL_LORENTZ:
                    if "rho" in want:
                        mo["rho"] = z()
                    if "J0" in want:
                        mo["J"] = [z(), z(), z()]
                    if "F0" in want:
                        mo["F"] = [z(), z(), z()]
                    if eng and "eng" in want:
                        mo["eng"] = z()
                elif kind == B.PL_DUST:
                    if "rho" in want:
                        mo["rho"] = z()
                    if "F0" in want:
                        mo["F"] = [z(), z(), z()]
                self.moms.append(mo)
                self.mom_blocks.append(block)
                self._fill_item(i)
                # initial state: float64 positions and velocities -> current set
                w = torch.from_numpy(it.particles.w).to(self.dev)
                np0 = it.particles.n
                if weights:
                    sets[0]["w"][:np0].copy_(w.to(fdt))
                if ids:
                    sets[0]["id"][:np0].copy_(torch.from_numpy(it.particles.id.astype(np.int64)).to(self.dev))
            self.stream.synchronize()
        self.load_state([(it.particles.x, it.particles.u) for it in wl.items])

    # ------------------------------------------------------------------
    def _fill_item(self, i):
        it = self.wl.items[i]
        kind = KIND[self.wl.species[it.species].kind]
        rec = self.items[i]
        rec.box = it.box
        rec.species = it.species
        p = self.parts[i]
        rec.p.n = it.particles.n
        rec.p.cur = 0
        if p["eng"] is not None:
            rec.p.nbins = p["eng"][0].shape[1]
            for s in range(len(p["eng"])):
                rec.p.eng[s] = _ptr(p["eng"][s])
                rec.p.chi[s] = _ptr(p["chi"][s])
        for s, st in enumerate(p["sets"]):
            rec.p.cell[s] = _ptr(st["cell"])
            for a in range(3):
                rec.p.x[s][a] = _ptr(st["x"][a]) if a < self.ndim else None
                rec.p.u[s][a] = _ptr(st["u"][a])
            rec.p.w[s] = _ptr(st["w"])
            rec.p.id[s] = _ptr(st["id"])
        if p["fp"] is not None:
            for a in range(3):
                rec.p.fp[a] = _ptr(p["fp"][a])
        rec.p.tile_start = _ptr(p["tile_start"])
        rec.p.runs = _ptr(p["runs"])
        f = self.fields[it.box]
        for a in range(3):
            if kind == B.PL_LORENTZ:
                rec.f.E[a] = _ptr(f["E"][a])
                rec.f.B[a] = _ptr(f["B"][a])
            else:
                rec.f.vg[a] = _ptr(f["vg"][a])
            if "divu" in f:
                rec.f.B[a] = _ptr(f["B"][a])
                rec.f.vg[a] = _ptr(f["vg"][a])
        if "divu" in f:
            rec.f.divu = _ptr(f["divu"])
        mo = self.moms[i]
        rec.m.rho = _ptr(mo.get("rho"))
        for a in range(3):
            rec.m.J[a] = _ptr(mo["J"][a]) if "J" in mo else None
            rec.m.F[a] = _ptr(mo["F"][a]) if "F" in mo else None
        rec.m.eng = _ptr(mo.get("eng"))

    def load_state(self, states):
        """Write float64 (x, u) numpy pairs into every item's current set."""
        torch = self.torch
        worst = B.PL_OK
        for i, (x, u) in enumerate(states):
            xd = [torch.from_numpy(np.ascontiguousarray(x[a])).to(self.dev) for a in range(3)]
            ud = [torch.from_numpy(np.ascontiguousarray(u[a])).to(self.dev) for a in range(3)]
            torch.cuda.synchronize()
            B.pl_part_pack(self.ctx, self.items[i], [t.data_ptr() for t in xd[: self.ndim]],
                           [t.data_ptr() for t in ud])
            st = self.sync()
            worst = st if worst == B.PL_OK else worst
        self.load_status = worst
        return worst

    # ------------------------------------------------------------------
    def step(self, dt=None, flags=B.PL_FUSE_DEPOSIT | B.PL_ZERO_FIRST, items=None):
        dt = self.wl.dt if dt is None else dt
        arr = self.items if items is None else items
        return B.pl_part_gather_push(self.ctx, arr, dt, flags)

    def deposit(self, flags=B.PL_ZERO_FIRST):
        return B.pl_part_deposit(self.ctx, self.items, flags)

    def sort(self):
        return B.pl_part_sort(self.ctx, self.items)

    def spectra(self, dt=None, cr=1e-4, u_rad=0.0, ub=0.5):
        dt = self.wl.dt if dt is None else dt
        return B.pl_part_spectra(self.ctx, self.items, dt, cr, u_rad, ub)

    def boundary(self, open_dims, ghost):
        """Delete particles outside the active cells of the open dimensions and
        compact; returns the number removed per item."""
        return B.pl_part_boundary(self.ctx, self.items, open_dims, ghost)[1]

    def inject(self, i, x, u, w=None, ids=None, eng=None, chi=None):
        """Append particles to item i from float64 numpy arrays x, u (3, k)."""
        torch = self.torch
        k = x.shape[1]
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev) if a is not None else None
        xd = [dev(x[a]) for a in range(3)]
        ud = [dev(u[a]) for a in range(3)]
        wd, idd = dev(w), dev(ids.astype(np.int64) if ids is not None else None)
        ed, cd = dev(eng), dev(chi)
        torch.cuda.synchronize()
        ptr = lambda t: t.data_ptr() if t is not None else None
        st = B.pl_part_inject(self.ctx, self.items[i], k, [ptr(t) for t in xd[: self.ndim]], [ptr(t) for t in ud],
                              ptr(wd), ptr(idd), ptr(ed), ptr(cd), cap=self.capacity[i])
        self.stream.synchronize()
        return st

    def spectra_state(self, i):
        """(eng, chi) of item i's current set as (n, nbins) float64 numpy arrays."""
        self.stream.synchronize()
        cur = self.items[i].p.cur
        n = self.items[i].p.n
        return self.parts[i]["eng"][cur][:n].cpu().numpy(), self.parts[i]["chi"][cur][:n].cpu().numpy()

    def sync(self):
        return B.pl_part_sync(self.ctx)

    def sums(self):
        return B.pl_part_sums(self.ctx, self.items)

    def state(self, i):
        """(x, u, id) of item i as float64 numpy arrays (current set)."""
        torch = self.torch
        n = int(self.items[i].p.n)
        with torch.cuda.stream(self.stream):
            x = [torch.zeros(n, dtype=torch.float64, device=self.dev) for _ in range(3)]
            u = [torch.zeros(n, dtype=torch.float64, device=self.dev) for _ in range(3)]
        self.stream.synchronize()
        B.pl_part_unpack(self.ctx, self.items[i], [t.data_ptr() for t in x[: self.ndim]], [t.data_ptr() for t in u])
        st = self.sync()
        cur = self.items[i].p.cur
        ids = self.parts[i]["sets"][cur]["id"]
        xs = np.stack([t.cpu().numpy() for t in x])
        us = np.stack([t.cpu().numpy() for t in u])
        idn = ids[:n].cpu().numpy().astype(np.uint64) if ids is not None else None
        return xs, us, idn, st

    def raw(self, i):
        """Current-set device tensors of item i (cell, x, u, w, id) as numpy."""
        cur = self.items[i].p.cur
        st = self.parts[i]["sets"][cur]
        self.stream.synchronize()
        out = {}
        for k, v in st.items():
            if v is None:
                continue
            out[k] = [t.cpu().numpy() for t in v] if isinstance(v, list) else v.cpu().numpy()
        out["tile_start"] = self.parts[i]["tile_start"].cpu().numpy()
        if self.parts[i]["runs"] is not None:
            out["runs"] = self.parts[i]["runs"].cpu().numpy()
        return out

    def moments(self, i):
        self.stream.synchronize()
        mo = self.moms[i]
        out = {}
        for k, v in mo.items():
            out[k] = [t.cpu().numpy() for t in v] if isinstance(v, list) else v.cpu().numpy()
        return out

    def zero_moments(self):
        """Zero every item's moment grids on the context's stream."""
        with self.torch.cuda.stream(self.stream):
            for blk in self.mom_blocks:
                blk.zero_()

    def close(self):
        if self.ctx:
            B.pl_part_finalize(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
