// Evaluation of one system: neighbour list (rebuilt by the skin rule), T message-passing
// layers forward, then the hand-written reverse sweep for forces and virial.
//
// Forward (Sec. 2.1, Eqs. (1)-(2)): for t = 0..T-1 the edge pass gives S^t of the locals;
// for t < T-1 the message NN of each element gives c^{t+1} of the locals and the ghost
// copies receive their owners' values (the per-layer exchange of Sec. 2.2); the energy NN
// of S^{T-1}'s densities gives E_i, summed in FP64.
// Backward (Sec. 2.2, Eqs. (3)-(5)): Sbar^{T-1} from the energy NN's VJP; for t = T-1..0
// the edge adjoint adds forces and virial and, for t >= 1, the message adjoints cbar^t of
// every ext atom, which are summed onto their owners (the reverse exchange) and pulled
// through the message NN of layer t-1 to give Sbar^{t-1}.  dc^0/dr = 0 ends the sweep.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "runtime.hpp"

#include <rocprofiler-sdk-roctx/roctx.h>

namespace reann {

NNLayout nn_layout(int F, int H, int nh, int out) {
    NNLayout l;
    int prev = F;
    int64_t o = 0;
    for (int k = 0; k <= nh; ++k) {
        const int d = (k == nh) ? out : H;
        l.w_off.push_back(o); o += (int64_t)d * prev;
        l.b_off.push_back(o); o += d;
        l.din.push_back(prev);
        l.dout.push_back(d);
        prev = d;
    }
    l.size = o;
    return l;
}

static void upload(DevBuf &b, const std::vector<double> &v, bool to_float, hipStream_t st) {
    const size_t n = v.size() ? v.size() : 1;
    if (to_float) {
        std::vector<float> f(n, 0.f);
        for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
        b.ensure(n * 4);
        HIP_OK(hipMemcpyAsync(b.p, f.data(), n * 4, hipMemcpyHostToDevice, st));
        HIP_OK(hipStreamSynchronize(st));
    } else {
        b.ensure(n * 8);
        if (v.size()) HIP_OK(hipMemcpyAsync(b.p, v.data(), v.size() * 8, hipMemcpyHostToDevice, st));
        HIP_OK(hipStreamSynchronize(st));
    }
}

DeviceWeights &Model::weights(int device, hipStream_t st) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = dev.find(device);
    if (it != dev.end()) return *it->second;
    auto w = std::make_unique<DeviceWeights>();
    upload(w->msg64, msg, false, st);
    upload(w->en64, en, false, st);
    upload(w->c064, c0, false, st);
    upload(w->msg32, msg, true, st);
    upload(w->en32, en, true, st);
    upload(w->c032, c0, true, st);
    auto &ref = *w;
    dev[device] = std::move(w);
    return ref;
}

const MfmaSet &Model::mfma(int device, hipStream_t st, bool energy, OpType op) {
    DeviceWeights &w = weights(device, st);
    std::lock_guard<std::mutex> lk(mu);
    auto &slot = w.mf[energy ? 1 : 0][(int)op];
    if (slot) return *slot;
    auto set = std::make_unique<MfmaSet>();
    const NNLayout &lay = energy ? en_nn : msg_nn;
    const std::vector<double> &blob = energy ? en : msg;
    const int count = energy ? n_species : (T_max - 1) * n_species;
    // host: padded FP32 copies of every matrix, then one device conversion per matrix
    std::vector<float> host;
    std::vector<size_t> foff;          // float offset of each padded matrix in `host`
    std::vector<int> rows_, cols_, lds_;
    std::vector<float> scales;
    for (int q = 0; q < count; ++q)
        for (int k = 0; k < nh; ++k) {
            const double *W = blob.data() + (size_t)q * lay.size + lay.w_off[k];
            const int dout = lay.dout[k], din = lay.din[k];
            for (int dir = 0; dir < 2; ++dir) {
                const int r = dir == 0 ? dout : din, cdim = dir == 0 ? din : dout, ld = pad_k(cdim);
                foff.push_back(host.size());
                rows_.push_back(r); cols_.push_back(cdim); lds_.push_back(ld);
                double amax = 0;
                for (int a = 0; a < r; ++a)
                    for (int b = 0; b < ld; ++b) {
                        double v = 0;
                        if (b < cdim) v = dir == 0 ? W[(size_t)a * din + b] : W[(size_t)b * din + a];
                        host.push_back((float)v);
                        amax = std::max(amax, std::fabs(v));
                    }
                scales.push_back(op == OpType::FP8 ? (amax > 0 ? (float)(amax / 448.0) : 1.0f) : 1.0f);
                const int idx = (int)scales.size() - 1;
                if (dir == 0) { set->sc_fwd.push_back(idx); set->ld_fwd.push_back(ld); }
                else { set->sc_bwd.push_back(idx); set->ld_bwd.push_back(ld); }
            }
        }
    DevBuf tmp;
    tmp.ensure(std::max<size_t>(host.size(), 1) * 4);
    if (!host.empty()) HIP_OK(hipMemcpyAsync(tmp.p, host.data(), host.size() * 4, hipMemcpyHostToDevice, st));
    set->scales.ensure(std::max<size_t>(scales.size(), 1) * 4);
    if (!scales.empty()) HIP_OK(hipMemcpyAsync(set->scales.p, scales.data(), scales.size() * 4, hipMemcpyHostToDevice, st));
    const size_t eb = op_bytes(op);
    set->buf.ensure(std::max<size_t>(host.size(), 1) * eb);
    for (size_t i = 0; i < foff.size(); ++i) {
        const size_t ob = foff[i] * eb;
        convert_operand(st, op, tmp.as<float>() + foff[i], rows_[i], cols_[i], lds_[i], set->buf.as<char>() + ob,
                        lds_[i], set->scales.as<float>() + i);
        if (i % 2 == 0) set->off_fwd.push_back(ob);
        else set->off_bwd.push_back(ob);
    }
    HIP_OK(hipStreamSynchronize(st));
    slot = std::move(set);
    return *slot;
}

bool Model::on_device(int device, int prec) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = dev.find(device);
    if (it == dev.end()) return false;
    if (prec == REANN_FP64) return true;
    auto has = [&](OpType o) { return it->second->mf[0][(int)o] && it->second->mf[1][(int)o]; };
    if (prec == REANN_FP8)   // the FP8 rung also calibrates in FP32 and runs its adjoint in BF16
        return has(OpType::FP8) && has(OpType::F32) && has(OpType::BF16);
    return has(prec == REANN_BF16 ? OpType::BF16 : OpType::F32);
}

EdgeConsts Model::edge_consts() const {
    EdgeConsts e{};
    for (int m = 0; m < K; ++m) {
        e.centres[m] = centres[m];
        e.alphas[m] = alphas[m];
        e.alphas2[m] = alphas[m] * 1.4426950408889634;   // log2(e)
    }
    e.r_c = r_c;
    e.rc2 = r_c * r_c;
    e.ang_scale = ang_scale;
    return e;
}

DensityConsts Model::density_consts() const {
    DensityConsts d{};
    auto fact = [](int v) { double f = 1; for (int k = 2; k <= v; ++k) f *= k; return f; };
    int k = 0;
    for (int l = 0; l <= L; ++l) {
        d.lstart[l] = k;
        for (int lx = l; lx >= 0; --lx)
            for (int ly = l - lx; ly >= 0; --ly) {
                const int lz = l - lx - ly;
                d.w[k++] = fact(l) / (fact(lx) * fact(ly) * fact(lz));
            }
    }
    d.lstart[L + 1] = k;
    return d;
}

// -------------------------------------------------------------------- plan --

Plan::~Plan() {
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (check_ev) (void)hipEventDestroy(check_ev);
}

void Plan::init(Ctx *c_, Model *mm, const int32_t *spec, int64_t nn, const double cell_[9], const int32_t pbc_[3],
                int TT, const reann_opts *opt) {
    ctx = c_;
    m = mm;
    model_id = mm->id;
    if (nn <= 0) fail(REANN_E_INVALID, "n must be > 0");
    if (TT < 1 || TT > m->T_max) fail(REANN_E_INVALID, "T must be in [1, T_max]");
    T = TT;
    prec = opt ? opt->precision : REANN_FP32;
    if (prec != REANN_FP64 && prec != REANN_FP32 && prec != REANN_BF16 && prec != REANN_FP8)
        fail(REANN_E_INVALID, "unknown precision");
    fp64 = prec == REANN_FP64;
    op = prec == REANN_BF16 ? OpType::BF16 : (prec == REANN_FP8 ? OpType::FP8 : OpType::F32);
    if (op == OpType::FP8 && m->form != REANN_FORM_REANN)
        fail(REANN_E_UNSUPPORTED, "this message form runs in FP64, FP32 or BF16");
    const int exch = opt ? opt->exchange : REANN_EXCHANGE_MESSAGES;
    if (exch != REANN_EXCHANGE_MESSAGES && exch != REANN_EXCHANGE_NODE_FEATURES)
        fail(REANN_E_INVALID, "unknown exchange");
    nodefeat = exch == REANN_EXCHANGE_NODE_FEATURES;
    if (nodefeat && op == OpType::FP8) fail(REANN_E_UNSUPPORTED, "node-feature exchange runs in FP64, FP32 or BF16");
    rs = fp64 ? 8 : 4;
    skin = opt ? opt->skin : 0.0;
    if (!(skin >= 0.0) || !std::isfinite(skin)) fail(REANN_E_INVALID, "skin must be >= 0");
    for (int a = 0; a < 3; ++a) P[a] = (opt && opt->decomp[a] > 0) ? opt->decomp[a] : 1;
    std::memcpy(cell, cell_, sizeof cell);
    std::memcpy(pbc, pbc_, sizeof pbc);
    geom_init(g, cell, pbc, P, m->r_c, skin);
    n = nn;
    species.assign(spec, spec + nn);
    for (int64_t i = 0; i < n; ++i)
        if (species[i] < 0 || species[i] >= m->n_species) fail(REANN_E_INVALID, "species out of range");
    hipStream_t st = ctx->stream;
    int32_t *ds = d_species.resize(n);
    HIP_OK(hipMemcpyAsync(ds, species.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    m->weights(ctx->device, st);
    if (!fp64) {
        m->mfma(ctx->device, st, false, op);
        m->mfma(ctx->device, st, true, op);
        if (op == OpType::FP8)   // calibration forward in FP32, adjoint in BF16
            for (bool e : {false, true}) {
                m->mfma(ctx->device, st, e, OpType::F32);
                m->mfma(ctx->device, st, e, OpType::BF16);
            }
    }
    fp8s.ensure(16);
    fp8tmp.ensure(16);
}

bool Plan::same_system(const Model *mm, const int32_t *spec, int64_t nn, const double cell_[9], const int32_t pbc_[3],
                       int TT, const reann_opts *opt) const {
    // the id, not only the address: a model created after this plan's model was freed can
    // have the same address (m itself is not read, it may be dangling)
    if (mm != m || mm->id != model_id || nn != n || TT != T) return false;
    const int pr = opt ? opt->precision : REANN_FP32;
    const double sk = opt ? opt->skin : 0.0;
    const bool nf = opt && opt->exchange == REANN_EXCHANGE_NODE_FEATURES;
    if (pr != prec || sk != skin || nf != nodefeat) return false;
    for (int a = 0; a < 3; ++a) {
        const int pa = (opt && opt->decomp[a] > 0) ? opt->decomp[a] : 1;
        if (pa != P[a] || (pbc_[a] != 0) != (pbc[a] != 0)) return false;
    }
    if (std::memcmp(cell_, cell, sizeof cell) != 0) return false;
    return std::memcmp(spec, species.data(), nn * sizeof(int32_t)) == 0;
}

// Phase names for the trace markers (the order of the Phase enumeration).
static const char *const kPhaseName[REANN_N_PHASES] = {"reann: nlist",      "reann: edge forward", "reann: density",
                                                        "reann: NN forward", "reann: ghost exchange", "reann: NN adjoint",
                                                        "reann: density adjoint", "reann: edge adjoint (centre)",
                                                        "reann: edge adjoint (gather)", "reann: other"};

void Plan::mark(hipStream_t st, int phase, int nlaunch) {
    // a host-side trace marker at the end of every phase's launches (rocprofv3 --marker-trace
    // shows them beside the kernels); no cost without a tracing tool
    if (phase >= 0 && phase < REANN_N_PHASES) roctxMarkA(kPhaseName[phase]);
    if (!timing) return;
    if (nev == ev.size()) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        ev.push_back(e);
        ev_phase.push_back(-1);
    }
    HIP_OK(hipEventRecord(ev[nev], st));
    ev_phase[nev] = phase;
    if (phase >= 0 && phase < REANN_N_PHASES) launches[phase] += nlaunch;
    ++nev;
}

int64_t Plan::collect_timing(double *ms, int64_t *nlaunch) {
    for (int q = 0; q < REANN_N_PHASES; ++q) ms[q] = 0.0;
    if (nev > 0) HIP_OK(hipEventSynchronize(ev[nev - 1]));
    for (size_t i = 1; i < nev; ++i) {
        const int ph = ev_phase[i];
        if (ph < 0 || ph >= REANN_N_PHASES) continue;
        float t = 0;
        HIP_OK(hipEventElapsedTime(&t, ev[i - 1], ev[i]));
        ms[ph] += t;
    }
    if (nlaunch)
        for (int q = 0; q < REANN_N_PHASES; ++q) nlaunch[q] = launches[q];
    const int64_t steps = timed_steps;
    nev = 0;
    timed_steps = 0;
    for (int q = 0; q < REANN_N_PHASES; ++q) launches[q] = 0;
    return steps;
}

// whether both atomic NNs run as fused kernels (FP32 or BF16 operands, supported widths)
bool Plan::fused() const {
    // the fused kernels form the paired density (or, at L = 0, take the radial form's sums)
    return !fp64 && m->form != REANN_FORM_DIAG && fused_nn_ok(op, m->F, m->H, m->nh, m->K, m->NL * m->K) &&
           fused_nn_ok(op, m->F, m->H, m->nh, 1, m->NL * m->K);
}

void Plan::alloc_buffers() {
    const int K = m->K, NL = m->NL, F = m->F, H = m->H, nh = m->nh;
    const int64_t ne = nl.n_ext;
    p4.ensure(ne * 32);
    const int64_t ns = nS();
    c.ensure((size_t)T * ne * K * rs);
    S.ensure((size_t)T * ns * NL * K * rs);
    if (!fused() && !radial()) rho.ensure((size_t)T * ns * F * rs);
    Z.ensure((size_t)T * nh * ns * H * rs);
    if (!fused()) Hh.ensure((size_t)2 * ns * H * rs);
    y.ensure((size_t)n * K * rs);
    ybar.ensure((size_t)n * rs);
    Eat.ensure((size_t)n * 8);
    Epart.ensure((size_t)(grid_for(n, 256) + 1) * 8);
    Sbar.ensure((size_t)ns * NL * K * rs);
    if (!fused() && !radial()) rhobar.ensure((size_t)ns * F * rs);
    if (radial()) cbar_next.ensure((size_t)ns * K * rs);
    if (!fused()) {
        const int wmax = F > H ? F : H;
        gA.ensure((size_t)ns * wmax * rs);
        gB.ensure((size_t)ns * wmax * rs);
    }
    cbar.ensure((size_t)ne * K * rs);
    this->F.ensure((size_t)ne * 3 * rs);
    Wpart.ensure((size_t)T * (edge_backward_blocks(ne) + 1) * 9 * 8);   // per layer, summed once
    disp.ensure(1025 * 8);
    col2.ensure((size_t)(nl.n_pairs + 1) * 4);
    fslot.ensure((size_t)(nl.n_pairs + 1) * 4);
    cpos.ensure((size_t)(nl.n_pairs + 1) * 4);
    rslot.ensure((size_t)(nl.n_pairs + 1) * 4);
    erec.ensure((size_t)(nl.n_pairs + 1) * edge_record_elems(K) * rs);
    nloc.ensure((size_t)(ne + 1) * 4);
    ngh.ensure((size_t)(ne + 1) * 4);
}

size_t Plan::device_bytes() const {
    size_t b = 0;
    for (const DevBuf *d : {&p4, &c, &S, &rho, &Z, &Hh, &y, &ybar, &Eat, &Epart, &Sbar, &rhobar, &gA, &gB,
                            &cbar, &F, &Wpart, &disp, &col2, &fslot, &cpos, &rslot, &nloc, &ngh, &erec, &fp8s,
                            &fp8tmp, &cbar_next})
        b += d->bytes;
    b += nl.perm.bytes() + nl.inv_perm.bytes() + nl.q.bytes() + nl.gh_owner.bytes() + nl.gh_shift.bytes() +
         nl.copy_ptr.bytes() + nl.copy_idx.bytes() + nl.row.bytes() + nl.col.bytes() + nl.rev.bytes() + nl.spec_ext.bytes() +
         nl.xref.bytes() + d_species.bytes();
    return b;
}

bool Plan::list_stale(const double *d_pos, hipStream_t st) {
    if (!built) return true;
    double d2 = 0;
    max_displacement2(st, nl, d_pos, disp.as<double>());
    HIP_OK(hipMemcpyAsync(&d2, disp.p, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    check_deferred();
    const double half = 0.5 * skin;
    return !(d2 <= half * half);
}

void Plan::rebuild(const double *d_pos, hipStream_t st, bool defer_check) {
    build_nlist(st, d_pos, d_species.ptr(), n, m->n_species, g, m->r_c, skin, nl, ns, nodefeat, defer_check);
    built = true;
    ++rebuilds;
    alloc_buffers();
    if (fp8_fused() && !fp8_ready) calibrate_fp8(d_pos, st);
}

int Plan::nn_ranges(int s, bool energy, int64_t (&a)[2], int64_t (&rows)[2]) const {
    a[0] = nl.seg[s];
    rows[0] = nl.seg[s + 1] - nl.seg[s];
    if (energy || !nodefeat) return 1;
    a[1] = nl.gseg[s];
    rows[1] = nl.gseg[s + 1] - nl.gseg[s];
    return 2;
}

int Plan::nn_forward(hipStream_t st, int t, bool energy) {
    DeviceWeights &w = m->weights(ctx->device, st);
    const NNLayout &lay = energy ? m->en_nn : m->msg_nn;
    const char *blob = energy ? (fp64 ? w.en64.as<char>() : w.en32.as<char>())
                              : (fp64 ? w.msg64.as<char>() : w.msg32.as<char>());
    const int F = m->F, H = m->H, nh = m->nh, K = m->K;
    int nfused = 0;
    std::vector<FusedNN> segs;   // the fused kernel's segments, launched together below
    for (int s = 0; s < m->n_species; ++s) {
      int64_t ra[2], rn[2];
      const int nr = nn_ranges(s, energy, ra, rn);
      for (int q = 0; q < nr; ++q) {
        const int64_t a = ra[q], rows = rn[q];
        if (rows <= 0) continue;
        const int64_t nn_index = energy ? s : (int64_t)t * m->n_species + s;
        const char *p = blob + (size_t)nn_index * lay.size * rs;
        const char *A = featptr(t) + (size_t)a * F * rs;
        int lda = F;
        const bool f8 = fp8_fused();
        const MfmaSet *mf = fp64 ? nullptr : (f8 ? fp8set[energy ? 1 : 0].get() : &m->mfma(ctx->device, st, energy, op));
        char *out = energy ? y.as<char>() + (size_t)a * rs : cptr(t + 1) + (size_t)a * K * rs;
        const int dout = energy ? 1 : K;
        if (fused()) {
            FusedNN f{};
            f.rows = rows; f.F = F; f.H = H; f.nh = nh; f.dout = dout;
            f.L = m->L; f.K = K; f.dc = m->density_consts();
            f.S = (const float *)(Sptr(t) + (size_t)a * m->NL * K * rs);
            for (int k = 0; k < nh; ++k) {
                const size_t qi = (size_t)nn_index * nh + k;
                f.W[k] = mf->buf.as<char>() + mf->off_fwd[qi];
                f.ldw[k] = mf->ld_fwd[qi];
                f.b[k] = (const float *)(p + lay.b_off[k] * rs);
                f.Z[k] = (float *)(Zptr(t, k) + (size_t)a * H * rs);
                f.zscale[k] = f8 ? fp8_zscale[energy ? 1 : 0][qi] : 1.0f;
                f.hinv[k] = f8 ? fp8_hinv[energy ? 1 : 0][qi] : 1.0f;
            }
            f.xinv = f8 ? fp8_xinv[energy ? 1 : 0].as<float>() + (size_t)nn_index * F : nullptr;
            f.ldz = H;
            f.Wout = (const float *)(p + lay.w_off[nh] * rs);
            f.bout = (const float *)(p + lay.b_off[nh] * rs);
            if (energy) {   // the energy readout takes its weights and bias in FP64
                const double *p64 = w.en64.as<double>() + (size_t)nn_index * lay.size;
                f.Wout64 = p64 + lay.w_off[nh];
                f.bout64 = p64 + lay.b_off[nh];
            }
            f.C = (float *)out; f.ldc = dout;
            segs.push_back(f);
            continue;
        }
        for (int k = 0; k < nh; ++k) {
            char *Zk = Zptr(t, k) + (size_t)a * H * rs;
            char *Hk = Hptr(t, k) + (size_t)a * H * rs;
            if (fp64) {
                dense(st, fp64, EPI_BIAS_SILU, true, rows, lay.din[k], H, A, lda, p + lay.w_off[k] * rs,
                      p + lay.b_off[k] * rs, Zk, H, Hk, H);
            } else {
                const size_t qi = (size_t)nn_index * nh + k;
                if (op == OpType::FP8)
                    amax_scale(st, (const float *)A, rows, lay.din[k], lda, fp8s.as<float>(), fp8tmp.as<uint32_t>());
                gemm_mfma(st, op, EPI_BIAS_SILU, rows, lay.din[k], H, (const float *)A, lda,
                          mf->buf.as<char>() + mf->off_fwd[qi], mf->ld_fwd[qi], (const float *)(p + lay.b_off[k] * rs),
                          (float *)Zk, H, (float *)Hk, H, fp8s.as<float>(), mf->scales.as<float>() + mf->sc_fwd[qi]);
            }
            A = Hk;
            lda = H;
        }
        if (fp64)
            dense(st, fp64, EPI_BIAS, true, rows, H, dout, A, lda, p + lay.w_off[nh] * rs, p + lay.b_off[nh] * rs,
                  nullptr, 0, out, dout);
        else if (energy) {   // FP64 weights and bias, as in the fused kernel
            const double *p64 = w.en64.as<double>() + (size_t)nn_index * lay.size;
            out_layer_energy(st, rows, H, (const float *)A, lda, p64 + lay.w_off[nh], p64 + lay.b_off[nh], (float *)out,
                             dout);
        } else
            out_layer_fwd(st, rows, H, dout, (const float *)A, lda, (const float *)(p + lay.w_off[nh] * rs),
                          (const float *)(p + lay.b_off[nh] * rs), (float *)out, dout);
      }
    }
    // the elements' rows (and ghosts') are independent: one launch over all of them
    if (!segs.empty()) nfused += mlp_fused_segments(st, op, true, segs.data(), (int)segs.size());
    return nfused;
}

// VJP of the NN applied at layer t (energy NN if `energy`), from output adjoint gout
// [n][ldg] to Sbar when the NN is fused (the density adjoint included), else to rhobar.
int Plan::nn_vjp(hipStream_t st, int t, bool energy, const char *gout, int ldg) {
    DeviceWeights &w = m->weights(ctx->device, st);
    const NNLayout &lay = energy ? m->en_nn : m->msg_nn;
    const char *blob = energy ? (fp64 ? w.en64.as<char>() : w.en32.as<char>())
                              : (fp64 ? w.msg64.as<char>() : w.msg32.as<char>());
    const int F = m->F, H = m->H, nh = m->nh;
    int nfused = 0;
    std::vector<FusedNN> segs;   // the fused kernel's segments, launched together below
    OpType seg_op = op;
    for (int s = 0; s < m->n_species; ++s) {
      int64_t ra[2], rn[2];
      const int nr = nn_ranges(s, energy, ra, rn);
      for (int q = 0; q < nr; ++q) {
        const int64_t a = ra[q], rows = rn[q];
        if (rows <= 0) continue;
        const int64_t nn_index = energy ? s : (int64_t)t * m->n_species + s;
        const char *p = blob + (size_t)nn_index * lay.size * rs;
        // output layer: zbar_{nh-1} = (gout W_out) * silu'(Z_{nh-1})
        const char *gin = gout + (size_t)a * ldg * rs;
        int ldin = ldg;
        char *bufs[2] = {gA.as<char>(), gB.as<char>()};
        int cur = 0;
        // the FP8 rung's adjoint takes BF16 operands (the forward's FP8 scales are calibrated
        // for activations, not for their adjoints)
        const OpType bop = fp8_fused() ? OpType::BF16 : op;
        const MfmaSet *mf = fp64 ? nullptr : &m->mfma(ctx->device, st, energy, bop);
        if (fused()) {
            FusedNN f{};
            f.rows = rows; f.F = F; f.H = H; f.nh = nh; f.dout = lay.dout[nh];
            f.L = m->L; f.K = m->K; f.dc = m->density_consts();
            f.S = (const float *)(Sptr(t) + (size_t)a * m->NL * m->K * rs);
            for (int k = 0; k < nh; ++k) {
                const size_t qi = (size_t)nn_index * nh + k;
                f.W[k] = mf->buf.as<char>() + mf->off_bwd[qi];
                f.ldw[k] = mf->ld_bwd[qi];
                f.Z[k] = (float *)(Zptr(t, k) + (size_t)a * H * rs);
            }
            f.ldz = H;
            f.Wout = (const float *)(p + lay.w_off[nh] * rs);
            f.G = (const float *)gin; f.ldg = ldin;
            f.C = (float *)(Sbar.as<char>() + (size_t)a * m->NL * m->K * rs); f.ldc = m->NL * m->K;
            segs.push_back(f);
            seg_op = bop;
            continue;
        }
        for (int k = nh; k >= 1; --k) {
            char *dst = bufs[cur] + (size_t)a * H * rs;
            const char *Zk = Zptr(t, k - 1) + (size_t)a * H * rs;
            if (fp64) {
                dense(st, fp64, EPI_DSILU, false, rows, lay.dout[k], lay.din[k], gin, ldin, p + lay.w_off[k] * rs,
                      nullptr, (void *)Zk, H, dst, H);
            } else if (k == nh) {   // the output layer's adjoint has few inputs
                out_layer_vjp(st, rows, lay.dout[k], lay.din[k], (const float *)gin, ldin,
                              (const float *)(p + lay.w_off[k] * rs), (const float *)Zk, H, (float *)dst, H);
            } else {
                const size_t qi = (size_t)nn_index * nh + k;
                if (op == OpType::FP8)
                    amax_scale(st, (const float *)gin, rows, lay.dout[k], ldin, fp8s.as<float>(), fp8tmp.as<uint32_t>());
                gemm_mfma(st, op, EPI_DSILU, rows, lay.dout[k], lay.din[k], (const float *)gin, ldin,
                          mf->buf.as<char>() + mf->off_bwd[qi], mf->ld_bwd[qi], nullptr, (float *)Zk, H, (float *)dst, H,
                          fp8s.as<float>(), mf->scales.as<float>() + mf->sc_bwd[qi]);
            }
            gin = dst;
            ldin = H;
            cur ^= 1;
        }
        // radial form: dE/dx is dE/dS (F = K, S is [n][1][K])
        char *rb = (radial() ? Sbar.as<char>() : rhobar.as<char>()) + (size_t)a * F * rs;
        if (fp64) {
            dense(st, fp64, EPI_NONE, false, rows, lay.dout[0], F, gin, ldin, p + lay.w_off[0] * rs, nullptr, nullptr, 0,
                  rb, F);
        } else {
            const size_t qi = (size_t)nn_index * nh;
            if (op == OpType::FP8)
                amax_scale(st, (const float *)gin, rows, lay.dout[0], ldin, fp8s.as<float>(), fp8tmp.as<uint32_t>());
            gemm_mfma(st, op, EPI_NONE, rows, lay.dout[0], F, (const float *)gin, ldin, mf->buf.as<char>() + mf->off_bwd[qi],
                      mf->ld_bwd[qi], nullptr, nullptr, 0, (float *)rb, F, fp8s.as<float>(),
                      mf->scales.as<float>() + mf->sc_bwd[qi]);
        }
      }
    }
    if (!segs.empty()) nfused += mlp_fused_segments(st, seg_op, false, segs.data(), (int)segs.size());
    return nfused;
}

bool Plan::prepare(const double *d_pos, hipStream_t st) {
    const bool stale = list_stale(d_pos, st);
    if (stale) rebuild(d_pos, st);
    else if (fp8_fused() && !fp8_ready) calibrate_fp8(d_pos, st);
    return stale;
}

// FP8 calibration (once, on the plan's first evaluation): an FP32 forward gives every NN's
// inputs; per NN, the largest |rho| over its element's rows and features sets the scale of the
// density input, s = headroom max|rho| / 448 (one scale per tensor; the kernels take one per
// feature, folded into layer 0's operand W_0 diag(s), but per-feature scales measured no better:
// e4m3's error here is its 3-bit mantissa, not its range), and the largest |SiLU(z)| of each
// hidden layer sets that layer's input scale.  Weights are stored in FP8 with one scale per
// matrix.  The headroom of 2 keeps values up to twice the calibration maximum in range; larger
// ones saturate at 448.  The scales stay fixed afterwards (a trajectory keeps its ranges).
void Plan::calibrate_fp8(const double *d_pos, hipStream_t st) {
    constexpr double kHeadroom = 2.0;
    const int F = m->F, H = m->H, nh = m->nh, ns = m->n_species, K = m->K;
    const OpType saved = op;
    const uint64_t gen = generation;
    op = OpType::F32;
    DevBuf tmpE;
    launch_forward(d_pos, static_cast<double *>(tmpE.ensure(64)), nullptr, st);
    op = saved;
    generation = gen;   // the calibration pass is not one of the caller's forwards
    const int nmsg = (m->T_max - 1) * ns, nen = ns;
    const int nq[2] = {nmsg, nen};
    DevBuf amax;
    const size_t na = (size_t)(nmsg + nen) * (F + nh);
    float *dam = static_cast<float *>(amax.ensure(std::max<size_t>(na, 1) * 4));
    zero(st, dam, std::max<size_t>(na, 1) * 4);
    const DensityConsts dc = m->density_consts();
    auto slot = [&](int e, int q) { return dam + ((size_t)(e ? nmsg : 0) + q) * (F + nh); };
    for (int t = 0; t < T; ++t) {
        const bool energy = t == T - 1;
        for (int s = 0; s < ns; ++s) {
            const int64_t a = nl.seg[s], rows = nl.seg[s + 1] - nl.seg[s];
            if (rows <= 0) continue;
            const int q = energy ? s : t * ns + s;
            float *out = slot(energy, q);
            density_absmax(st, m->L, K, rows, dc, (const float *)(Sptr(t) + (size_t)a * m->NL * K * rs), out);
            for (int k = 0; k + 1 < nh; ++k)
                silu_absmax(st, rows, H, H, (const float *)(Zptr(t, k) + (size_t)a * H * rs), out + F + k);
        }
    }
    std::vector<float> ham(std::max<size_t>(na, 1));
    HIP_OK(hipMemcpyAsync(ham.data(), dam, ham.size() * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int e = 0; e < 2; ++e) {
        const NNLayout &lay = e ? m->en_nn : m->msg_nn;
        const std::vector<double> &blob = e ? m->en : m->msg;
        const int count = nq[e];
        auto set = std::make_unique<MfmaSet>();
        std::vector<float> host, xinv((size_t)std::max(count, 1) * F, 1.0f), scales;
        std::vector<size_t> foff;
        std::vector<int> rows_, cols_, lds_;
        fp8_zscale[e].assign((size_t)std::max(count, 1) * nh, 1.0f);
        fp8_hinv[e].assign((size_t)std::max(count, 1) * nh, 1.0f);
        for (int q = 0; q < count; ++q) {
            const float *am = ham.data() + ((size_t)(e ? nmsg : 0) + q) * (F + nh);
            double rmax = 0.0;
            for (int f = 0; f < F; ++f) rmax = std::max(rmax, (double)am[f]);
            std::vector<double> sx(F, kHeadroom * (rmax > 0.0 ? rmax : 1.0) / 448.0);
            for (int f = 0; f < F; ++f) xinv[(size_t)q * F + f] = (float)(1.0 / sx[f]);
            for (int k = 0; k < nh; ++k) {
                const double *W = blob.data() + (size_t)q * lay.size + lay.w_off[k];
                const int dout = lay.dout[k], din = lay.din[k], ld = pad_k(din);
                const double sig = k == 0 ? 1.0 : kHeadroom * (am[F + k - 1] > 0.0f ? am[F + k - 1] : 1.0) / 448.0;
                foff.push_back(host.size());
                rows_.push_back(dout); cols_.push_back(din); lds_.push_back(ld);
                double wmax = 0.0;
                for (int o = 0; o < dout; ++o)
                    for (int i = 0; i < ld; ++i) {
                        const double v = i < din ? W[(size_t)o * din + i] * (k == 0 ? sx[i] : 1.0) : 0.0;
                        host.push_back((float)v);
                        wmax = std::max(wmax, std::fabs(v));
                    }
                const double wsc = wmax > 0.0 ? wmax / 448.0 : 1.0;
                scales.push_back((float)wsc);
                set->off_fwd.push_back(0);
                set->ld_fwd.push_back(ld);
                fp8_zscale[e][(size_t)q * nh + k] = (float)(wsc * sig);
                fp8_hinv[e][(size_t)q * nh + k] = (float)(1.0 / sig);
            }
        }
        DevBuf tmp;
        tmp.ensure(std::max<size_t>(host.size(), 1) * 4);
        if (!host.empty()) HIP_OK(hipMemcpyAsync(tmp.p, host.data(), host.size() * 4, hipMemcpyHostToDevice, st));
        set->scales.ensure(std::max<size_t>(scales.size(), 1) * 4);
        if (!scales.empty())
            HIP_OK(hipMemcpyAsync(set->scales.p, scales.data(), scales.size() * 4, hipMemcpyHostToDevice, st));
        set->buf.ensure(std::max<size_t>(host.size(), 1));
        for (size_t i = 0; i < foff.size(); ++i) {
            convert_operand(st, OpType::FP8, tmp.as<float>() + foff[i], rows_[i], cols_[i], lds_[i],
                            set->buf.as<char>() + foff[i], lds_[i], set->scales.as<float>() + i);
            set->off_fwd[i] = foff[i];   // one byte per element: the byte offset equals the float offset
        }
        float *dx = static_cast<float *>(fp8_xinv[e].ensure(xinv.size() * 4));
        HIP_OK(hipMemcpyAsync(dx, xinv.data(), xinv.size() * 4, hipMemcpyHostToDevice, st));
        HIP_OK(hipStreamSynchronize(st));
        fp8set[e] = std::move(set);
    }
    fp8_ready = true;
}

namespace {
// A host-side trace range over a scope (closed on every exit, exceptions included).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};
}  // namespace

void Plan::forward(const double *d_pos, double *d_energy, double *d_atom_energy, hipStream_t st) {
    TraceRange range("reann: forward");
    mark(st, -1);
    if (auto_list && built && !(fp8_fused() && !fp8_ready)) {
        // The skin check goes to the device with the forward on the list it checks behind it,
        // and its answer is read while that forward runs, so the device does not wait for the
        // host between the check and the forward.  A stale list is rebuilt and the forward
        // enqueued again: its outputs are written again, in stream order.  (On a stale list
        // the first forward only misses pairs; every index it uses is the old list's own.)
        max_displacement2(st, nl, d_pos, disp.as<double>());
        double *h = check_host.get_double();
        HIP_OK(hipMemcpyAsync(h, disp.p, 8, hipMemcpyDeviceToHost, st));
        if (!check_ev) HIP_OK(hipEventCreateWithFlags(&check_ev, hipEventDisableTiming));
        HIP_OK(hipEventRecord(check_ev, st));
        mark(st, PH_NLIST, 0);
        launch_forward(d_pos, d_energy, d_atom_energy, st);
        HIP_OK(hipEventSynchronize(check_ev));
        check_deferred();
        const double half = 0.5 * skin;
        if (*h <= half * half) return;
        rebuild(d_pos, st);
        mark(st, PH_NLIST, 1);
        launch_forward(d_pos, d_energy, d_atom_energy, st);
        return;
    }
    const bool rebuilt = auto_list ? prepare(d_pos, st) : false;
    mark(st, PH_NLIST, rebuilt ? 1 : 0);
    launch_forward(d_pos, d_energy, d_atom_energy, st);
}

void Plan::launch_forward(const double *d_pos, double *d_energy, double *d_atom_energy, hipStream_t st) {
    if (!built) fail(REANN_E_STATE, "neighbour list not built");
    const int K = m->K;
    DeviceWeights &w = m->weights(ctx->device, st);
    refresh_positions(st, nl, d_pos, p4.as<double4>());
    // c^0 depends on the element alone and nothing writes it afterwards: set once per list build
    if (c0_build != rebuilds) {
        init_messages(st, fp64, nl.n_ext, K, nl.spec_ext.ptr(), fp64 ? w.c064.p : w.c032.p, cptr(0));
        c0_build = rebuilds;
    }
    EdgeArgs ea{n, nl.n_ext, nl.row.ptr(), nl.col.ptr(), p4.as<double4>()};
    CutList cl = cutlist();
    compact_cutoff(st, ea, m->r_c, cl);
    const EdgeConsts ec = m->edge_consts();
    const DensityConsts dc = m->density_consts();
    mark(st, PH_OTHER);
    for (int t = 0; t < T; ++t) {
        edge_forward(st, fp64, m->L, K, ea, cl, ec, cptr(t), Sptr(t));
        mark(st, PH_EDGE_FWD, 1);
        // node-feature exchange: the ghosts' orbital sums come from their owners, and the
        // message NN then runs over the ghosts as well
        const bool ghost_nn = nodefeat && t < T - 1;
        if (ghost_nn) {
            ghost_gather(st, fp64, n, nl.n_gh, m->NL * K, nl.gh_owner.ptr(), Sptr(t));
            mark(st, PH_GHOST);
        }
        if (!fused() && !radial()) {   // the fused NN kernels contract S themselves
            if (m->form == REANN_FORM_DIAG)
                density_sq(st, fp64, m->L, K, ghost_nn ? nl.n_ext : n, dc, Sptr(t), rhoptr(t));
            else
                density(st, fp64, m->L, K, ghost_nn ? nl.n_ext : n, dc, Sptr(t), rhoptr(t));
            mark(st, PH_DENSITY, 1);
        }
        if (t < T - 1) {
            mark(st, PH_NN_FWD, nn_forward(st, t, false));
            if (radial()) {   // c^{t+1} = c^t + NN(x^t) for the rows the NN ran over
                add_into(st, fp64, nS() * K, cptr(t + 1), cptr(t));
                mark(st, PH_OTHER);
            }
            if (!nodefeat) {
                ghost_gather(st, fp64, n, nl.n_gh, K, nl.gh_owner.ptr(), cptr(t + 1));
                mark(st, PH_GHOST);
            }
        }
    }
    mark(st, PH_NN_FWD, nn_forward(st, T - 1, true));
    energy_total(st, fp64, n, m->energy_scale, y.p, nl.perm.ptr(), have_ew ? d_ew.ptr() : nullptr, d_atom_energy,
                 Epart.as<double>(), d_energy);
    mark(st, PH_OTHER);
    have_forward = true;
    ++generation;
}

void Plan::backward(const double *d_g, double *d_forces, double *d_virial, hipStream_t st) {
    if (!have_forward) fail(REANN_E_STATE, "backward called before forward");
    TraceRange range("reann: backward");
    const int K = m->K;
    EdgeArgs ea{n, nl.n_ext, nl.row.ptr(), nl.col.ptr(), p4.as<double4>()};
    const CutList cl = cutlist();
    const EdgeConsts ec = m->edge_consts();
    const DensityConsts dc = m->density_consts();
    mark(st, -1);
    // the energy adjoints, and the force accumulator cleared, in one launch
    fill_energy_seed(st, fp64, n, m->energy_scale, d_g, nl.perm.ptr(), have_ew ? d_ew.ptr() : nullptr, ybar.p,
                     nl.n_ext * 3, this->F.p);
    mark(st, PH_OTHER);
    mark(st, PH_NN_BWD, nn_vjp(st, T - 1, true, ybar.as<char>(), 1));
    if (!fused() && !radial()) {
        if (m->form == REANN_FORM_DIAG) density_sq_vjp(st, fp64, m->L, K, n, dc, Sptr(T - 1), rhobar.p, Sbar.p);
        else density_vjp(st, fp64, m->L, K, n, dc, Sptr(T - 1), rhobar.p, Sbar.p);
        mark(st, PH_DENSITY_ADJ, 1);
    }
    // the centre role's per-block virial partials of the T layers side by side, summed once
    int nbw = 0;
    for (int t = T - 1; t >= 0; --t) {
        const int nb = edge_adjoint_centre(st, fp64, m->L, K, ea, cl, ec, cptr(t), Sbar.p, t > 0, this->F.p,
                                           Wpart.as<double>() + (size_t)nbw * 9, erec.p);
        nbw += nb;
        mark(st, PH_ADJ_CENTRE, 1);
        edge_adjoint_gather(st, fp64, K, ea, cl, t > 0, t == T - 1, erec.p, this->F.p, cbar.p);
        mark(st, PH_ADJ_GATHER, 1);
        if (t > 0) {
            // message exchange: the ghosts' message adjoints go back to their owners here;
            // node-feature exchange: the ghosts keep theirs (their message NN ran locally) and
            // the adjoints of their orbital sums go back after the NN's VJP
            if (!nodefeat) {
                ghost_reduce(st, fp64, n, K, nl.copy_ptr.ptr(), nl.copy_idx.ptr(), cbar.p);
                mark(st, PH_GHOST);
            }
            if (radial()) {   // c^t also reaches E through c^{t+1} = c^t + NN(x^t) (t < T - 1)
                if (t < T - 1) add_into(st, fp64, nS() * K, cbar.p, cbar_next.p);
                if (t > 1) copy_into(st, fp64, nS() * K, cbar_next.p, cbar.p);
                mark(st, PH_OTHER);
            }
            mark(st, PH_NN_BWD, nn_vjp(st, t - 1, false, cbar.as<char>(), K));
            if (!fused() && !radial()) {
                if (m->form == REANN_FORM_DIAG)
                    density_sq_vjp(st, fp64, m->L, K, nS(), dc, Sptr(t - 1), rhobar.p, Sbar.p);
                else
                    density_vjp(st, fp64, m->L, K, nS(), dc, Sptr(t - 1), rhobar.p, Sbar.p);
                mark(st, PH_DENSITY_ADJ, 1);
            }
            if (nodefeat) {   // the ghosts' dE/dS^{t-1} summed onto their owners
                ghost_reduce(st, fp64, n, m->NL * K, nl.copy_ptr.ptr(), nl.copy_idx.ptr(), Sbar.p);
                mark(st, PH_GHOST);
            }
        }
    }
    ghost_reduce(st, fp64, n, 3, nl.copy_ptr.ptr(), nl.copy_idx.ptr(), this->F.p);
    mark(st, PH_GHOST);
    // the seed carried g; forces are -dE/dx already scaled; the virial partials are summed in the
    // same launch
    forces_out(st, fp64, n, this->F.p, nl.perm.ptr(), nullptr, d_forces, Wpart.as<double>(), nbw, d_virial);
    mark(st, PH_OTHER);
    if (timing) ++timed_steps;
}

void Plan::get(int what, int t, double *host) {
    if (!have_forward) fail(REANN_E_STATE, "no forward has run");
    HIP_OK(hipDeviceSynchronize());   // the forward may have run on a caller's stream
    const int K = m->K, NL = m->NL;
    std::vector<int32_t> perm(n);
    HIP_OK(hipMemcpy(perm.data(), nl.perm.ptr(), n * 4, hipMemcpyDeviceToHost));
    if (what == 2) {
        std::vector<double> y_(n);
        if (fp64) HIP_OK(hipMemcpy(y_.data(), y.p, n * 8, hipMemcpyDeviceToHost));
        else {
            std::vector<float> f(n);
            HIP_OK(hipMemcpy(f.data(), y.p, n * 4, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i) y_[i] = f[i];
        }
        for (int64_t i = 0; i < n; ++i) host[perm[i]] = m->energy_scale * y_[i];
        return;
    }
    if (t < 0 || t >= T) fail(REANN_E_INVALID, "layer out of range");
    const int width = what == 0 ? NL * K : K;
    const char *src = what == 0 ? Sptr(t) : cptr(t);
    if (what != 0 && what != 1) fail(REANN_E_INVALID, "unknown quantity");
    std::vector<double> v((size_t)n * width);
    if (fp64) HIP_OK(hipMemcpy(v.data(), src, (size_t)n * width * 8, hipMemcpyDeviceToHost));
    else {
        std::vector<float> f((size_t)n * width);
        HIP_OK(hipMemcpy(f.data(), src, (size_t)n * width * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < f.size(); ++i) v[i] = f[i];
    }
    for (int64_t i = 0; i < n; ++i)
        std::memcpy(host + (size_t)perm[i] * width, v.data() + (size_t)i * width, width * 8);
}

}  // namespace reann
