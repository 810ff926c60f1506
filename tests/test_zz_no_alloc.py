"""The no-allocation interpolation entry point against the allocating one.

interpolate_to_particles_noalloc carves its scratch from the library's fixed
per-device region: on two calls in a row through the C-ABI (the second with
fewer particles and fewer entries, so stale contents of the first call sit
in the region) its values equal interpolate_to_particles' bit for bit (same
kernels, same summation order) and a sample matches the oracle within the
interpolation bar (1e-12 times the largest entry value); the context's own
workspace does not grow; a call that needs more than the region is refused
before anything runs."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed(pkg, ctx, workloads, n, seed, r_part):
    pos, m, h, rho = workloads.make_cloud("turbulent", n, seed=seed)
    src = pos[workloads.densest_particle(rho)][None, :]
    ps = pkg.build_pseudo_particles(ctx, pos, h, m, src, r_part=r_part, theta=0.5)
    return pos, ps


def test_noalloc_matches_allocating_entry_point(workloads, oracle):
    import paper_2410_15227_amd as pkg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = pkg.Context(0)
    ref_ctx = pkg.Context(0)
    try:
        held0 = ctx.workspace_info()["held"]
        for n, seed, r_part, k in ((60000, 61, 0.15, 3), (9000, 62, 0.1, 1)):
            say(f"case: no-alloc interpolation, turbulent {n} (seed {seed}), {k} component(s)")
            pos, ps = mixed(pkg, ref_ctx, workloads, n, seed, r_part)
            ne = ps["kind"].shape[0]
            g = np.random.default_rng(seed)
            vals = g.uniform(-1.0, 2.0, size=(ne, k)) if k > 1 else g.uniform(-1.0, 2.0, size=ne)
            xyz = torch.tensor(pos, device="cuda")
            out = torch.empty((n, k) if k > 1 else n, dtype=torch.float64, device="cuda")
            out.fill_(np.nan)
            got = pkg.interpolate_to_particles(ctx, xyz, ps, vals, out=out, noalloc=True)
            want = pkg.interpolate_to_particles(ref_ctx, xyz, ps, vals)
            torch.cuda.synchronize()
            assert torch.equal(got, want)
            sample = g.choice(n, 400, replace=False)
            own = ps["owner"].cpu().numpy()
            o = oracle.interpolate(pos[sample], own[sample], ps["xyz"].cpu().numpy(), ps["h"].cpu().numpy(),
                                   ps["kind"].cpu().numpy(), vals)
            err = np.abs(got.cpu().numpy()[sample] - o).max() / np.abs(vals).max()
            say(f"entries {ne}: identical to the allocating call; oracle sample max rel {err:.2e}")
            assert err <= 1e-12
        # the fixed region carried both calls: the context's workspace did not grow
        assert ctx.workspace_info()["held"] == held0
        # a call needing more than the region is refused before it runs
        with pytest.raises(pkg.SphmapError) as e:
            pkg._native.lib()  # loaded
            ctx.check(pkg._native.lib().interpolate_to_particles_noalloc(
                ctx.handle, 8_000_000, pkg._ptr(xyz), pkg._ptr(ps["owner"]), 1_000_000, pkg._ptr(ps["xyz"]),
                pkg._ptr(ps["h"]), pkg._ptr(ps["kind"]), pkg._ptr(torch.zeros(1, device="cuda")), 1,
                pkg._ptr(out), None))
        assert e.value.code == -1 and "fixed scratch" in str(e.value)
    finally:
        ctx.close()
        ref_ctx.close()
