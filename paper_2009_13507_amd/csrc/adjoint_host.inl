// adjoint_host.inl -- host side of the real-time adjoint (included by ssgp.hip).

template <typename R>
static int adjoint_steps(ssgp_grid g, const void *states, void *lam, int nsteps) {
    if (so_y_terms(g->p.so) && g->p.gamma != 0.0)
        return fail(SSGP_EINVAL, "the adjoint supports SO forms with x derivatives only");
    SSGP_TRY(build_tables<R>(g, MODE_ADJ));
    const int rows = g->dim == 2 ? g->ny : 1;
    // per-row dL/dOmega partials of every step of the call, then the step sums
    SSGP_TRY(g->adj_partials.ensure(sizeof(double) * ((size_t)rows * nsteps + nsteps)));
    const size_t se = (size_t)3 * plane_of(*g);
    const long long n0 = g->step_index - nsteps;
    Tables<R> &T = tables<R>(g);
    const int Lx = x_chunk(g->nx);
    const YShape ys = y_shape(g->ny);
    for (int k = nsteps - 1; k >= 0; --k) {
        const long long n = n0 + k;
        const double omega = omega_at(*g, n);
        if (g->dim == 2) {
            YArgs<R> ya = y_args<R>(g, MODE_ADJ, lam, nullptr);
            SSGP_TRY(launch_y<R>(*g, ya, ys));
        }
        AdjXArgs<R> a{};
        a.lam = static_cast<cx<R> *>(lam);
        a.psi_n = static_cast<const cx<R> *>(states) + (size_t)k * se;
        a.nx = g->nx;
        a.ny = rows;
        a.plane = plane_of(*g);
        a.dx = (R)g->dx;
        a.dy = (R)(g->dim == 2 ? g->dy : 0.0);
        a.x0 = (R)(-0.5 * g->nx * g->dx);
        a.y0 = (R)(g->dim == 2 ? -0.5 * g->ny * g->dy : 0.0);
        a.m = model<R>(*g, MODE_REAL, omega);
        a.cx_ = T.x[MODE_ADJ].coef();
        a.rdiag = T.x[MODE_ADJ].rdiag;
        XArgs<R> tmp{};
        fill_so<R>(tmp, *g, MODE_ADJ);
        for (int q = 0; q < 9; ++q) a.qx[q] = tmp.qx[q];
        a.qxmask = tmp.qxmask;
        a.omega_partials = g->adj_partials.as<double>() + (size_t)k * rows;
        LAUNCH_TRY(launch_adj_xpass<R>(lc(*g), a, Lx, rows));
    }
    double *partials = g->adj_partials.as<double>();
    LAUNCH_TRY(launch_omega_accumulate(lc(*g), partials, rows, nsteps, partials + (size_t)rows * nsteps, n0,
                                       g->steps_per_seg, (int)g->omega_sched.size(), g->omega_acc.as<double>()));
    g->step_index = n0;
    return SSGP_OK;
}
