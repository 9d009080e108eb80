"""The x sweep of a field split into x-slabs, as the distributed solver runs
it (Sec. 3.2): per block of lines, the forward shares slab after slab, each
handing its last x-plane of eliminated values to the next, then the backward
shares back, each handing its first x-plane of solution values to the
previous.  On one GPU the slabs are separate device arrays; with one stream
per slab and an event per (slab, block), slab r works on block b while slab
r + 1 works on block b - 1, as the processes would.  Launch order and
dependencies only: the arithmetic is the library's (bfvm_xslab_forward,
bfvm_xslab_backward)."""


def chained_x_sweep(grid, slabs, xb, lb, streams=None):
    """Sweep x through the slabs in place.

    grid:    the Grid of the whole domain (its Thomas constants at global x);
    slabs:   CUDA tensors, slab r holding x in [xb[r], xb[r + 1]) as
             [nz][ny][xb[r+1] - xb[r]][S] of the grid's dtype;
    xb:      slab bounds 0 = xb[0] < ... < xb[P] = nx;
    lb:      line-block bounds 0 = lb[0] < ... < lb[NB] = ny * nz * S;
    streams: one torch.cuda.Stream per slab, or None for the current stream
             (the shares then run one after another).
    Returns after enqueueing; the current stream waits for every slab."""
    import torch
    P = len(slabs)
    if len(xb) != P + 1 or xb[0] != 0 or xb[-1] != grid.nx:
        raise ValueError("xb must bound the slabs from 0 to nx")
    nl = grid.ny * grid.nz * grid.nsub
    if lb[0] != 0 or lb[-1] != nl:
        raise ValueError("lb must bound the line blocks from 0 to ny * nz * S")
    if streams is not None and grid._explicit_stream:
        raise ValueError("a grid bound to its own stream cannot follow the slab streams")
    cdt = torch.float32 if grid.dtype == "f32fast" else torch.float64
    fwd = [torch.empty(nl, dtype=cdt, device="cuda") for _ in range(P)]
    bwd = [torch.empty(nl, dtype=cdt, device="cuda") for _ in range(P)]
    main = torch.cuda.current_stream()
    if streams is None:
        streams = [main] * P
    start = torch.cuda.Event()
    start.record(main)
    for s in set(streams):
        s.wait_event(start)
    NB = len(lb) - 1
    done_f = [[torch.cuda.Event() for _ in range(NB)] for _ in range(P)]
    done_b = [[torch.cuda.Event() for _ in range(NB)] for _ in range(P)]
    for b in range(NB):
        l0, l1 = lb[b], lb[b + 1]
        for r in range(P):
            with torch.cuda.stream(streams[r]):
                if r > 0:
                    streams[r].wait_event(done_f[r - 1][b])
                grid.xslab_forward(slabs[r], xb[r], xb[r + 1], l0, l1, fwd[r - 1][l0:] if r > 0 else None,
                                   fwd[r][l0:])
                done_f[r][b].record(streams[r])
    for b in range(NB):
        l0, l1 = lb[b], lb[b + 1]
        for r in reversed(range(P)):
            with torch.cuda.stream(streams[r]):
                streams[r].wait_event(done_b[r + 1][b] if r < P - 1 else done_f[r][b])
                grid.xslab_backward(slabs[r], xb[r], xb[r + 1], l0, l1, bwd[r + 1][l0:] if r < P - 1 else None,
                                    bwd[r][l0:])
                done_b[r][b].record(streams[r])
    # the carry arrays were allocated on the current stream, which now waits
    # for every slab: their memory is reused only after the work using it
    for s in set(streams):
        main.wait_stream(s)
