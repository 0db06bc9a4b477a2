// Runtime objects behind the C ABI: model parameters on the device, a context (device +
// stream), and a plan that evaluates one system (neighbour list, layer buffers, kernels).
#pragma once

#include <atomic>
#include <map>
#include <memory>
#include <mutex>

#include "edge.hpp"
#include "mfma.hpp"
#include "mlp.hpp"
#include "nlist.hpp"

struct reann_model;
struct reann_ctx;
struct reann_plan;

namespace reann {

// One atomic NN inside a flat parameter blob: offsets of W_k and b_k (k = 0 .. nh).
struct NNLayout {
    std::vector<int64_t> w_off, b_off;
    std::vector<int> din, dout;
    int64_t size = 0;
};
NNLayout nn_layout(int F, int H, int nh, int out);

// Matrix-core operands of the hidden layers of every atomic NN: for NN q and hidden layer k,
// the forward operand W_k [dout][pad(din)] and the backward operand W_k^T [din][pad(dout)],
// in one operand type, with one scale per matrix (FP8: amax/448; otherwise 1).
struct MfmaSet {
    DevBuf buf, scales;
    std::vector<size_t> off_fwd, off_bwd;   // bytes, index q * nh + k
    std::vector<int> ld_fwd, ld_bwd;
    std::vector<int> sc_fwd, sc_bwd;        // index into scales
};

struct DeviceWeights {
    DevBuf msg64, en64, c064, msg32, en32, c032;
    std::unique_ptr<MfmaSet> mf[2][3];      // [msg, energy][OpType]
};

// A number no other model of this process has had: a freed model's address can be reused
// by the next one, so a plan cached for a system records the id of its model, not only the
// address.
inline uint64_t next_model_id() {
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}

struct Model {
    const uint64_t id = next_model_id();
    int n_species, L, K, T_max, nh, H, F, NL;
    int form = REANN_FORM_REANN;   // REANN_FORM_RADIAL: F = K features, residual message updates
    double r_c, ang_scale, energy_scale;
    std::vector<double> centres, alphas, c0, msg, en;
    NNLayout msg_nn, en_nn;
    std::mutex mu;
    std::map<int, std::unique_ptr<DeviceWeights>> dev;
    // device copy of the weights for `device` (created on first use)
    DeviceWeights &weights(int device, hipStream_t st);
    // matrix-core operands of the message (energy = false) or energy NNs for `op`
    const MfmaSet &mfma(int device, hipStream_t st, bool energy, OpType op);
    // whether the device copies an evaluation at `prec` reads already exist on `device`
    bool on_device(int device, int prec);
    EdgeConsts edge_consts() const;
    DensityConsts density_consts() const;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // plans and neighbour lists created on this context; reann_ctx_free defers the release
    // until the last of them is freed
    int users = 0;
    bool released = false;
    std::unique_ptr<struct Plan> cached;   // plan of the last host-API system
    const Model *cached_model = nullptr;
    DevBuf pos, forces, scal;
};

// timing phases (reann_plan_timing)
enum Phase {
    PH_NLIST = 0, PH_EDGE_FWD, PH_DENSITY, PH_NN_FWD, PH_GHOST, PH_NN_BWD, PH_DENSITY_ADJ, PH_ADJ_CENTRE,
    PH_ADJ_GATHER, PH_OTHER
};
static_assert(PH_OTHER + 1 == REANN_N_PHASES, "phase count");

struct Plan {
    Ctx *ctx = nullptr;
    Model *m = nullptr;
    uint64_t model_id = 0;   // m->id when the plan was made (m may since have been freed)
    int T = 1, prec = REANN_FP32;
    bool fp64 = false;
    size_t rs = 4;   // bytes of the working type
    Geom g{};
    int32_t P[3] = {1, 1, 1};
    double skin = 0, cell[9]{};
    int32_t pbc[3]{};
    int64_t n = 0;
    std::vector<int32_t> species;
    DArr<int32_t> d_species;
    NList nl;
    NListScratch ns;
    bool built = false;
    int64_t rebuilds = 0;
    int64_t c0_build = -1;   // the list build whose ext atoms cptr(0) holds c^0 for
    // layer buffers
    DevBuf p4, c, S, rho, Z, Hh, y, ybar, Eat, Epart, Sbar, rhobar, gA, gB, cbar, F, Wpart, disp, one;
    DevBuf cbar_next;                // radial form: dE/dc^{t+1} of the locals, carried by the residual
    DevBuf col2, fslot, cpos, rslot, nloc, ngh;   // in-cutoff compaction of the list for the current step
    DevBuf erec;                     // per-slot edge records of the adjoint
    DevBuf fp8s, fp8tmp;      // per-call activation scale for FP8 products
    OpType op = OpType::F32;
    bool have_forward = false;
    uint64_t generation = 0;   // forwards launched on this plan (reann_plan_generation)
    // weights of the atomic energies in E (caller order; reann_plan_set_energy_weights)
    DArr<double> d_ew;
    bool have_ew = false;
    // FP8 on the fused NN kernels: forward operands and scales calibrated on the plan's first
    // evaluation (see calibrate_fp8), per NN [message, energy] indexed like the weight blobs
    bool fp8_ready = false;
    std::unique_ptr<MfmaSet> fp8set[2];
    DevBuf fp8_xinv[2];                     // [NN][F] inverse per-feature scales of the density input
    std::vector<float> fp8_zscale[2], fp8_hinv[2];   // [NN * nh]
    bool timing = false;
    // events recorded at phase boundaries while timing is on; intervals are attributed to
    // the phase named by the event that closes them (phase -1: not attributed)
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_phase;
    size_t nev = 0;
    int64_t timed_steps = 0;
    int64_t launches[REANN_N_PHASES]{};

    ~Plan();
    void init(Ctx *c, Model *mm, const int32_t *spec, int64_t nn, const double cell_[9], const int32_t pbc_[3], int TT,
              const reann_opts *opt);
    bool same_system(const Model *mm, const int32_t *spec, int64_t nn, const double cell_[9], const int32_t pbc_[3],
                     int TT, const reann_opts *opt) const;
    void forward(const double *d_pos, double *d_energy, double *d_atom_energy, hipStream_t st);
    // skin check (one stream synchronisation) and rebuild if needed; true if rebuilt, in which
    // case device buffers may have moved
    bool prepare(const double *d_pos, hipStream_t st);
    // false: forwards neither check the skin rule nor rebuild (reann_plan_set_list_policy)
    bool auto_list = true;
    // the skin check of a forward on a built list: its result copied to the host, and the
    // event after the copy
    PinnedWord check_host;
    hipEvent_t check_ev = nullptr;
    // the two halves of prepare: the skin check alone (true if the list was never built or an
    // atom has moved more than skin/2 since), and the rebuild (with the FP8 calibration the
    // first time), which allocates
    bool list_stale(const double *d_pos, hipStream_t st);
    // defer_check: the list's last consistency check is read by check_deferred (after the
    // caller's next wait for the stream) instead of by a wait here
    void rebuild(const double *d_pos, hipStream_t st, bool defer_check = false);
    void check_deferred() { reann::check_deferred(ns); }
    // the forward's launches only: no synchronisation and no allocation, so it can be captured
    void launch_forward(const double *d_pos, double *d_energy, double *d_atom_energy, hipStream_t st);
    size_t device_bytes() const;
    void backward(const double *d_g, double *d_forces, double *d_virial, hipStream_t st);
    void get(int what, int t, double *host);
    // per-phase kernel time (ms) accumulated since the last call; returns the step count
    int64_t collect_timing(double *ms, int64_t *nlaunch);

    // the FP8 rung's NN forward runs on the fused kernels (calibrated operands); its adjoint
    // then takes the BF16 operands
    bool fp8_fused() const { return op == OpType::FP8 && fused(); }

  private:
    void calibrate_fp8(const double *d_pos, hipStream_t st);
    void alloc_buffers();
    char *cptr(int t) const { return c.as<char>() + (size_t)t * nl.n_ext * m->K * rs; }
    char *Sptr(int t) const { return S.as<char>() + (size_t)t * nS() * m->NL * m->K * rs; }
    char *rhoptr(int t) const { return rho.as<char>() + (size_t)t * nS() * m->F * rs; }
    bool radial() const { return m->form == REANN_FORM_RADIAL; }
    // node-feature exchange: ghosts carry their own S^t, Z and NN results for the message NNs
    bool nodefeat = false;
    int64_t nS() const { return nodefeat ? nl.n_ext : n; }   // rows of the per-layer NN buffers
    // the atomic NNs' input at layer t: the density, or for the radial form the sums S[0]
    // themselves (S is [n][1][K] there, the same layout as [n][F])
    char *featptr(int t) const { return radial() ? Sptr(t) : rhoptr(t); }
    char *Zptr(int t, int k) const { return Z.as<char>() + ((size_t)t * m->nh + k) * nS() * m->H * rs; }
    // hidden activations of the per-layer (unfused) path: two buffers used in turn
    char *Hptr(int, int k) const { return Hh.as<char>() + (size_t)(k & 1) * nS() * m->H * rs; }
    // row ranges (first row, count) an NN of element s runs over: its locals, and for the
    // message NNs under node-feature exchange its ghosts too
    int nn_ranges(int s, bool energy, int64_t (&a)[2], int64_t (&rows)[2]) const;
    bool fused() const;
    // both return the launches of the fused NN kernel (0 on the per-layer path)
    int nn_forward(hipStream_t st, int t, bool energy);
    int nn_vjp(hipStream_t st, int t, bool energy, const char *gout, int ldg);
    void mark(hipStream_t st, int phase, int nlaunch = 0);
    CutList cutlist() {
        return CutList{nl.row.ptr(),        col2.as<int32_t>(),  nloc.as<int32_t>(), ngh.as<int32_t>(),
                       fslot.as<int32_t>(), cpos.as<int32_t>(), rslot.as<int32_t>(), nl.rev.ptr()};
    }
};

}  // namespace reann

struct reann_model { reann::Model impl; };
struct reann_ctx { reann::Ctx impl; };
namespace reann {
void set_last_error(const std::string &msg);   // message returned by reann_last_error on this thread
void ctx_acquire(Ctx *c);
void ctx_release(Ctx *c);   // frees the context once released and unused
}
struct reann_plan { reann::Plan impl; };
