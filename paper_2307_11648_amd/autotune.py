"""Autotuned schedule of the single-target selection.

Columns are independent, so how one launch lays them out changes only the
speed, never a result.  Two choices are tuned, four schedules in all:

* the column order: the columns' natural order, or a spatial (Morton) order
  from csel_spatial_order, under which columns whose candidate pools overlap
  run side by side on an XCD and share its L2;
* the waves per column: one wavefront holding a column's whole pool, or the
  pool split over 2 (pools <= 128) or 4 (pools <= 512) wavefronts that
  exchange each pick's argmax through LDS (csel_select_and_factor_sched):
  fewer registers per wavefront, so more resident wavefronts.

Which schedule wins depends on the pool size, the precision and the point
cloud, so the first call for a shape class times each once on the stream it
runs on and keeps the fastest; later calls of the class reuse the choice.
Choices can persist in a JSON file, which a later process reads back.

The multi-target selection (csel_aggregated_select_sched) is tuned the same
way between one workgroup per group and a group's rows split over workgroups
of 256, 512 or 1,024 threads: these give bit-identical results.  Mixed runs
that the register-resident kernel covers keep it untuned (its FP32 arithmetic
is its own, so a different choice could change a near-tied pick).

The tuner only chooses between launches of the library's kernels; every step
of the selection runs in them.
"""
from __future__ import annotations

import json
import math
import os

from . import csel

SCHEDULES = ("natural", "spatial", "natural/mw", "spatial/mw")
AGG_SCHEDULES = ("one_group", "split256", "split512", "split1024")
_FORMAT_VERSION = 2


def shape_key(dim: int, two_nu: int, n_targets: int, stride: int, k: int, precision: str) -> str:
    """Shape class of a selection problem: the kernel instantiation it runs
    (pool rows per lane, pick capacity, precision, smoothness, dimension) and
    the column count to the nearest power of two."""
    rpl = 1 if stride <= 64 else 2 if stride <= 128 else 4 if stride <= 256 else 8
    kmax = 16 if k <= 16 else 32
    tb = max(0, int(math.ceil(math.log2(max(1, n_targets)))))
    return f"d{dim}/nu{two_nu}/pool{64 * rpl}/k{kmax}/{precision}/T2^{tb}"


def agg_shape_key(dim: int, two_nu: int, n_groups: int, stride: int, max_members: int, k: int, precision: str,
                  post_var: bool) -> str:
    """Shape class of a multi-target selection: group count and rows per group
    (pool + members) to the next power of two, members, picks, precision and
    whether posterior variances are asked for."""
    gb = max(0, int(math.ceil(math.log2(max(1, n_groups)))))
    rb = max(0, int(math.ceil(math.log2(max(1, stride + max_members)))))
    return f"agg/d{dim}/nu{two_nu}/G2^{gb}/rows2^{rb}/m{max_members}/k{k}/{precision}/pv{int(bool(post_var))}"


def check_permutation(order, n: int) -> None:
    """Raise ValueError unless `order` holds each of 0 .. n-1 exactly once:
    the spatial schedule writes only the columns it lists."""
    import torch

    if order.dim() != 1 or order.shape[0] != n:
        raise ValueError("order must hold every column once")
    o = order.to(torch.int64)
    if n and (bool((o < 0).any()) or bool((o >= n).any())
              or not bool((torch.bincount(o, minlength=n) == 1).all())):
        raise ValueError("order must be a permutation of the columns")


def _event_timer(run, stream):
    """Milliseconds of one call of `run` on `stream`, by HIP events recorded
    on that stream (the kernels are enqueued there)."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    run()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1)


class SelectTuner:
    """Chooses, per shape class, the faster column schedule of
    csel_select_and_factor.

    path        -- optional JSON file the choices are read from and written to
    min_columns -- below this many columns the natural order is used untimed
    timer       -- timer(run, stream) -> ms; HIP events by default
    """

    def __init__(self, path: str | None = None, min_columns: int = 4096, timer=None):
        self.path = path
        self.min_columns = int(min_columns)
        self._timer = timer or _event_timer
        self.choices: dict[str, dict] = {}
        self.tuning_runs = 0
        self._counts = {}
        if path and os.path.exists(path):
            self.choices = self._read(path)

    @staticmethod
    def _read(path: str) -> dict:
        try:
            with open(path) as f:
                doc = json.load(f)
        except (OSError, ValueError):
            return {}
        if not isinstance(doc, dict) or doc.get("version") != _FORMAT_VERSION:
            return {}
        ch = doc.get("choices", {})
        return {key: v for key, v in ch.items()
                if isinstance(v, dict) and v.get("schedule") in SCHEDULES + AGG_SCHEDULES}

    def save(self) -> None:
        if not self.path:
            return
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"version": _FORMAT_VERSION, "choices": self.choices}, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def choose(self, key: str, runners: dict, stream=None) -> str:
        """The recorded schedule of `key`, or, on its first use, the faster of
        `runners` (schedule name -> callable), each run once to warm up and
        once timed."""
        got = self.choices.get(key)
        if got is not None and got["schedule"] in runners:
            return got["schedule"]
        ms = {}
        for name, run in runners.items():
            run()
            ms[name] = float(self._timer(run, stream))
        self.tuning_runs += 1
        names = list(runners)
        best = min(ms, key=lambda name: (ms[name], names.index(name)))
        self.choices[key] = {"schedule": best, "ms": ms}
        self.save()
        return best

    def _count(self, n: int, device):
        import torch

        t = self._counts.get((n, str(device)))
        if t is None:
            t = torch.tensor([n], dtype=torch.int32, device=device)
            self._counts[(n, str(device))] = t
        return t

    def select_and_factor(self, points, kernel, targets, pool, pool_len, k: int, precision: str = "mixed",
                          order=None, out: dict | None = None, stream=None) -> dict:
        """csel_select_and_factor under the tuned schedule.  `order` is a
        spatial order of the columns (csel.spatial_order); without it, or for
        fewer than min_columns columns, the natural order runs."""
        T = targets.shape[0]
        if out is None:
            import torch

            dev = points.device
            out = {
                "sel": torch.empty((T, k), dtype=torch.int32, device=dev),
                "factor": torch.empty((T, k + 1), dtype=torch.float64, device=dev),
                "log_condvar": torch.empty(T, dtype=torch.float64, device=dev),
                "status": torch.empty(T, dtype=torch.uint8, device=dev),
            }
        if order is None or T < self.min_columns:
            return csel.select_and_factor(points, kernel, targets, pool, pool_len, k, precision, out=out,
                                          stream=stream)
        n_all = self._count(T, targets.device)
        stride = pool.shape[1] if pool.dim() == 2 else 0
        mw = csel.select_waves_per_column(stride)

        def natural():
            csel.select_and_factor(points, kernel, targets, pool, pool_len, k, precision, out=out, stream=stream)

        def spatial():
            csel.select_and_factor_list(points, kernel, targets, pool, pool_len, k, precision, order, n_all, T, out,
                                        stream=stream)

        def natural_mw():
            csel.select_and_factor_sched(points, kernel, targets, pool, pool_len, k, precision, waves=mw, out=out,
                                         stream=stream)

        def spatial_mw():
            csel.select_and_factor_sched(points, kernel, targets, pool, pool_len, k, precision, waves=mw,
                                         col_list=order, col_count=n_all, max_cols=T, out=out, stream=stream)

        key = shape_key(points.shape[1], int(kernel.two_nu), T, stride, k, precision)
        if key not in self.choices or order.shape[0] != T:
            check_permutation(order, T)  # once per shape class (it reads the order back)
        runners = {"natural": natural, "spatial": spatial, "natural/mw": natural_mw, "spatial/mw": spatial_mw}
        runners[self.choose(key, runners, stream)]()
        return out

    def aggregated_select(self, points, kernel, group_ptr, members, max_members: int, pool, pool_len, k: int,
                          precision: str = "fp64", want_factor: bool = False, want_post_var: bool = False,
                          want_gap: bool = False, out: dict | None = None, workspace=None, stream=None) -> dict:
        """csel_aggregated_select under the tuned schedule of its shape class
        (one workgroup per group, or split rows of 256, 512 or 1,024 threads;
        split rows only without factor output and for at most 1,024 groups)."""
        G = group_ptr.numel() - 1
        stride = pool.shape[1] if pool.dim() == 2 else 0
        args = (points, kernel, group_ptr, members, max_members, pool, pool_len, k, precision)
        kw = dict(want_factor=want_factor, want_post_var=want_post_var, want_gap=want_gap, stream=stream)
        register = (precision == "mixed" and not want_post_var and stride <= 512 and max_members <= 32 and k <= 64)
        if register or G == 0:
            return csel.aggregated_select(*args, out=out, workspace=workspace, **kw)
        out = csel.aggregated_select(*args, out=out, workspace=workspace, schedule="one_group", **kw)
        workspace = out["workspace"]
        key = agg_shape_key(points.shape[1], int(kernel.two_nu), G, stride, max_members, k, precision,
                            want_post_var)
        names = ["one_group"]
        if not want_factor and G <= 1024 and k <= 256 and max_members <= 128:
            names += ["split256", "split512", "split1024"]
        got = self.choices.get(key)
        if got is not None and got["schedule"] in names:
            return csel.aggregated_select(*args, out=out, workspace=workspace, schedule=got["schedule"], **kw)
        runners = {}
        for name in names:
            def run(name=name):
                csel.aggregated_select(*args, out=out, workspace=workspace, schedule=name, **kw)
            try:
                run()  # a split grid the device cannot hold is refused
            except csel.CselError:
                continue
            runners[name] = run
        runners[self.choose(key, runners, stream)]()
        return out
