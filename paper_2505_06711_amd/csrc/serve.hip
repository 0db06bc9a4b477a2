// Continuous-batching server for energy + force requests on many independent systems.
//
// Each registered system keeps its positions, velocities, last forces, skinned neighbour
// list and layer buffers resident on the device once admitted.  An engine thread keeps up
// to kSlots requests in flight, each on its own stream, so the steps of different systems
// overlap on the device; a request that arrives while others run is admitted as soon as a
// slot and HBM budget are free (budget exhausted: idle resident systems are evicted, least
// recently used first, else the request waits).  The engine only admits and completes
// requests; a pool of kWorkers launcher threads enqueues each admitted step on its slot's
// stream, so that a step that has to rebuild its neighbour list (several waits for the
// device) does not hold up the launches of the others.  A step is one HIP-graph replay of the
// captured forward + backward when the neighbour list is unchanged; the list is rebuilt and
// the graph re-captured when an atom has moved more than skin/2.  Every system has its own
// buffers and the kernels are deterministic, so a result does not depend on what else is in
// flight.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <random>
#include <shared_mutex>
#include <thread>

#include "runtime.hpp"

using namespace reann;

namespace {

constexpr int kSlots = 8;
constexpr int kWorkers = 4;
// energy, virial (9), kinetic energy, displacement^2, max |v_c|, max |a_c|, the displacement^2
// that the next drift of the same dt will give, one spare
constexpr int kOutHead = 16;
constexpr double kAccel = 9.648533212e-3;   // (eV/A) / amu in A/fs^2

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// The drift of one position component; the same function predicts it a step ahead, so the
// prediction and the drift agree to the last bit.
__device__ inline double drift(double x, double v, double F, double minv, double dt) {
    const double a = F * minv * kAccel;
    return x + v * dt + 0.5 * a * dt * dt;
}

__global__ void k_vv_drift(int64_t n, double dt, const int32_t *__restrict__ spec, const double *__restrict__ minv,
                           double *__restrict__ x, const double *__restrict__ v, const double *__restrict__ F) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 3) return;
    x[t] = drift(x[t], v[t], F[t], minv[spec[t / 3]], dt);
}

constexpr double kBoltzmann = 8.617333262e-5;   // eV / K
constexpr int kKeBlock = 256;

// Kinetic energy K = (1/2) sum m v^2 of one system in a fixed order: per-block partial sums of
// m v^2 over consecutive components (a tree in LDS), then one block sums the partials in
// block order.  The blocks also take the largest velocity and acceleration components
// (|v_c| and |F_c / m| in A/fs and A/fs^2).  When T0 > 0 and tau > 0 the final block forms the
// thermostat's velocity factor lambda (else 1): Berendsen, lambda^2 = 1 + (dt / tau)(T0 / T - 1)
// with T = 2 K / (3 n k_B); CSVR, lambda^2 = K' / K with K' the kinetic energy resampled from the
// host-drawn normal r1 and chi-square s (see include/reann.h).  It writes aux[0] = lambda and,
// to the result head, lambda^2 K (eV: the kinetic energy after the rescaling that k_vv_post
// applies), lambda max|v_c| and max|a_c|.
constexpr int kAuxKe = 16;       // kinetic partials, 3 per block

// The kick of a velocity-Verlet step with the new forces F, then the block's kinetic partials
// of the kicked velocities; the first thread also clears the two displacement maxima that
// k_vv_post raises.
__global__ __launch_bounds__(kKeBlock) void k_vv_kick_ke(int64_t n3, double dt, const int32_t *__restrict__ spec,
                                                          const double *__restrict__ minv, double *__restrict__ v,
                                                          const double *__restrict__ Fold, const double *__restrict__ F,
                                                          double *__restrict__ part, unsigned long long *__restrict__ dmax) {
    __shared__ double sh[3][kKeBlock];
    const int64_t t = (int64_t)blockIdx.x * kKeBlock + threadIdx.x;
    if (t == 0) dmax[0] = dmax[3] = 0ull;
    double s = 0.0, vm = 0.0, am = 0.0;
    if (t < n3) {
        const double mi = minv[spec[t / 3]];
        const double vt = v[t] + 0.5 * (Fold[t] + F[t]) * mi * kAccel * dt;
        v[t] = vt;
        if (mi > 0.0) {
            s = vt * vt / mi;
            vm = fabs(vt);
            am = fabs(F[t] * mi * kAccel);
        }
    }
    sh[0][threadIdx.x] = s; sh[1][threadIdx.x] = vm; sh[2][threadIdx.x] = am;
    __syncthreads();
    for (int h = kKeBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + h]);
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = sh[0][0]; part[3 * blockIdx.x + 1] = sh[1][0]; part[3 * blockIdx.x + 2] = sh[2][0];
    }
}

// From sum m v^2 (s2, amu A^2/fs^2), max |v_c| and max |a_c|: the kinetic energy, the thermostat's
// factor lambda (aux[0]) and the result head (see above).
__device__ inline void ke_thermostat(double s2, double vm, double am, int64_t n, double dt, double T0, double tau,
                                     int kind, const double *__restrict__ rng, double *__restrict__ aux,
                                     double *__restrict__ head) {
    const double K = 0.5 * s2 / kAccel;   // amu A^2 / fs^2 -> eV
    double lam2 = 1.0;
    if (T0 > 0.0 && tau > 0.0 && K > 0.0) {
        const double nf = 3.0 * (double)n;
        if (kind == REANN_THERMO_CSVR) {
            const double r1 = rng[0], s_chi2 = rng[1];
            const double K0 = 0.5 * nf * kBoltzmann * T0, c = exp(-dt / tau);
            const double Kn = K + (1.0 - c) * (K0 * (r1 * r1 + s_chi2) / nf - K) +
                              2.0 * r1 * sqrt(c * (1.0 - c) * K * K0 / nf);
            lam2 = fmax(0.0, Kn / K);
        } else {
            const double Tcur = 2.0 * K / (nf * kBoltzmann);
            lam2 = fmax(0.0, 1.0 + dt / tau * (T0 / Tcur - 1.0));
        }
    }
    const double lam = sqrt(lam2);
    aux[0] = lam;
    head[0] = lam2 * K;
    head[2] = lam * vm;
    head[3] = am;
}

__global__ __launch_bounds__(kKeBlock) void k_ke_final(int64_t n, int nb, double dt, double T0, double tau,
                                                        int kind, const double *__restrict__ rng,
                                                        double *__restrict__ aux, double *__restrict__ head) {
    __shared__ double sh[3][kKeBlock];
    const double *part = aux + kAuxKe;
    double s = 0.0, vm = 0.0, am = 0.0;
    for (int b = threadIdx.x; b < nb; b += kKeBlock) {
        s += part[3 * b];
        vm = fmax(vm, part[3 * b + 1]);
        am = fmax(am, part[3 * b + 2]);
    }
    sh[0][threadIdx.x] = s; sh[1][threadIdx.x] = vm; sh[2][threadIdx.x] = am;
    __syncthreads();
    for (int h = kKeBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + h]);
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) ke_thermostat(sh[0][0], sh[1][0], sh[2][0], n, dt, T0, tau, kind, rng, aux, head);
}

// A system of up to kKeOneBlock / 3 atoms: the kick, the kinetic energy and the thermostat in
// one block (thread t takes components t, t + kKeBlock, ... in order, then the tree).
constexpr int64_t kKeOneBlock = 3 * 8192;

__global__ __launch_bounds__(kKeBlock) void k_vv_kick_ke_one(int64_t n3, double dt, const int32_t *__restrict__ spec,
                                                              const double *__restrict__ minv, double *__restrict__ v,
                                                              const double *__restrict__ Fold, const double *__restrict__ F,
                                                              unsigned long long *__restrict__ dmax, double T0, double tau,
                                                              int kind, const double *__restrict__ rng,
                                                              double *__restrict__ aux, double *__restrict__ head) {
    __shared__ double sh[3][kKeBlock];
    if (threadIdx.x == 0) dmax[0] = dmax[3] = 0ull;
    double s = 0.0, vm = 0.0, am = 0.0;
    for (int64_t t = threadIdx.x; t < n3; t += kKeBlock) {
        const double mi = minv[spec[t / 3]];
        const double vt = v[t] + 0.5 * (Fold[t] + F[t]) * mi * kAccel * dt;
        v[t] = vt;
        if (mi > 0.0) {
            s += vt * vt / mi;
            vm = fmax(vm, fabs(vt));
            am = fmax(am, fabs(F[t] * mi * kAccel));
        }
    }
    sh[0][threadIdx.x] = s; sh[1][threadIdx.x] = vm; sh[2][threadIdx.x] = am;
    __syncthreads();
    for (int h = kKeBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + h]);
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) ke_thermostat(sh[0][0], sh[1][0], sh[2][0], n3 / 3, dt, T0, tau, kind, rng, aux, head);
}

// The bits of a non-negative double (or a NaN) as an unsigned integer: their order is the
// order of the values, with every NaN above +inf, so an integer atomic max takes the largest
// value (a NaN, from a blown-up system, counts as too far) in any order of arrival.
__device__ inline unsigned long long order_bits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ inline double nan_max2(double a, double b) { return (b > a || b != b) ? b : a; }

// After a step, one thread per atom: the new forces become the old ones, the positions and
// velocities go to the output block.  A velocity-Verlet step (vv) first rescales the velocities
// by aux[0] and raises dmax[0] to the squared largest displacement of an atom since the list
// was built (xref, in the list's local order) and dmax[3] to the same after the drift of dt
// that the next step would make (drift() on the final velocities and forces).
__global__ __launch_bounds__(256) void k_vv_post(int64_t n, double dt, const int32_t *__restrict__ spec,
                                                 const double *__restrict__ minv, const double *__restrict__ F,
                                                 double *__restrict__ Fold, const double *__restrict__ x,
                                                 double *__restrict__ xout, double *__restrict__ v,
                                                 double *__restrict__ vout, const double *__restrict__ aux, int vv,
                                                 const int32_t *__restrict__ inv_perm, const double *__restrict__ xref,
                                                 unsigned long long *__restrict__ dmax) {
    __shared__ double sh[2][256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double d2 = 0.0, p2 = 0.0;
    if (i < n) {
        const double lam = vv ? aux[0] : 1.0, mi = vv ? minv[spec[i]] : 0.0;
        const int64_t l = vv ? inv_perm[i] : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t t = 3 * i + c;
            const double f = F[t], xc = x[t];
            Fold[t] = f;
            xout[t] = xc;
            double vt = v[t];
            if (vv) {
                vt *= lam;
                v[t] = vt;
                const double r = xref[3 * l + c], dx = xc - r, dp = drift(xc, vt, f, mi, dt) - r;
                d2 += dx * dx;
                p2 += dp * dp;
            }
            vout[t] = vt;
        }
    }
    if (!vv) return;   // uniform over the grid
    sh[0][threadIdx.x] = d2;
    sh[1][threadIdx.x] = p2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] = nan_max2(sh[0][threadIdx.x], sh[0][threadIdx.x + h]);
            sh[1][threadIdx.x] = nan_max2(sh[1][threadIdx.x], sh[1][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(dmax, order_bits(sh[0][0]));
        atomicMax(dmax + 3, order_bits(sh[1][0]));
    }
}

__global__ void k_copy_d(int64_t n, const double *__restrict__ a, double *__restrict__ b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = a[t];
}

struct Sys {
    uint64_t id = 0;
    int64_t n = 0;
    std::vector<int32_t> species;
    double cell[9]{};
    int32_t pbc[3]{};
    std::vector<double> pos, vel, forces;   // host copies, authoritative while not resident
    bool have_forces = false;               // forces of the current positions are known
    // residency
    std::unique_ptr<Plan> plan;
    // d_out = [E, W (9), K, d^2, vmax, amax, d_next^2, 0, F (3n), positions (3n), velocities (3n)]:
    // the step writes E, W and F in place and the motion figures, positions and velocities after
    // it; the head and the wanted vectors are copied back to h_res
    DevBuf d_pos, d_vel, d_Fold, d_out, d_aux;   // d_aux: [lambda, ..., kinetic partials from kAuxKe]
    // motion after the last velocity-Verlet step (largest displacement since the list was
    // built, largest velocity and acceleration components): bound the next step's displacement
    // when its dt differs from the one predicted for, so that the skin check (a device round
    // trip) is needed only near the edge
    bool motion_known = false;
    double disp = 0, vmax = 0, amax = 0;
    // the displacement (since the list build) the next drift gives if it takes pred_dt
    bool pred_known = false;
    double pred = 0, pred_dt = 0;
    // caller positions the neighbour list was last built from, when that build came from an
    // EVAL request (host positions): later EVAL requests check the skin rule on the host
    std::vector<double> xref_h;
    bool xref_ok = false;
    double *E() { return d_out.as<double>(); }
    double *W() { return d_out.as<double>() + 1; }
    double *KE() { return d_out.as<double>() + 10; }
    double *F() { return d_out.as<double>() + kOutHead; }
    double *P() { return d_out.as<double>() + kOutHead + 3 * n; }
    double *V() { return d_out.as<double>() + kOutHead + 6 * n; }
    std::mt19937_64 rng;   // CSVR draws
    DArr<int32_t> d_spec;
    // pinned host buffers while resident: the step's results (d_out copied back) and the CSVR
    // draws of the step (copied to d_rng)
    double *h_res = nullptr, *h_rng = nullptr;
    DevBuf d_rng;
    // the step after the positions are in place as one HIP graph, captured for a request kind,
    // a time step, the vectors skipped and a neighbour-list build
    hipGraphExec_t tail = nullptr;
    int64_t tail_rebuilds = -1;
    bool tail_vv = false;
    int32_t tail_skip = 0;
    double tail_dt = 0.0;
    size_t bytes = 0;
    int64_t last_used = 0;
    bool busy = false;
    // set when a request of this system failed for its inputs: its device state was dropped
    // (it may have been half updated), and later requests for it fail with REANN_E_STATE
    std::string failed;
    void free_host() {
        if (h_res) (void)hipHostFree(h_res);
        if (h_rng) (void)hipHostFree(h_rng);
        h_res = h_rng = nullptr;
    }
    ~Sys() {
        if (tail) (void)hipGraphExecDestroy(tail);
        free_host();
    }
};

struct Req {
    uint64_t ticket = 0, sys = 0;
    int32_t kind = REANN_REQ_EVAL;
    double dt = 0;
    int32_t skip = 0;   // REANN_OUT_* vectors not brought back
    std::vector<double> pos;
    int64_t t_submit = 0;
};

struct Done {
    double energy = 0, virial[9]{}, kinetic = 0;
    std::vector<double> forces, positions, velocities;
    int32_t skip = 0;
    int64_t t_submit = 0, t_done = 0;
    reann_status status = REANN_OK;
    std::string error;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool active = false;              // engine: taken by a request
    // set by the launcher: kQueued until the step is enqueued and `ev` recorded (kLaunched), or
    // kFailed with the error in `err`
    std::atomic<int> state{0};
    std::string err;
    reann_status err_code = REANN_E_DEVICE;
    Req req;
    Sys *sys = nullptr;
};

// slot states: the launcher has the step (queued), enqueued it (launched), hit a device error
// (failed: fatal for the server), or refused it for its inputs (rejected: only that request
// fails, and its system is set aside)
constexpr int kQueued = 0, kLaunched = 1, kFailed = 2, kRejected = 3;

// Keeps HIP-graph captures apart from device allocation and release on the server's other
// threads: work that may allocate or free (making a system resident, evicting it, pinned
// result buffers, neighbour-list rebuilds) holds it shared, so such work runs concurrently; a
// capture (with the instantiation and the release of the graph it replaces) holds it
// exclusively.  A waiting capture bars new shared holders, so captures are not starved by a
// stream of rebuilds.
class CaptureGate {
    std::mutex m;
    std::condition_variable cv;
    int readers = 0, writers_waiting = 0;
    bool writer = false;

  public:
    void lock_shared() {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return !writer && writers_waiting == 0; });
        ++readers;
    }
    void unlock_shared() {
        std::lock_guard<std::mutex> lk(m);
        if (--readers == 0) cv.notify_all();
    }
    void lock() {
        std::unique_lock<std::mutex> lk(m);
        ++writers_waiting;
        cv.wait(lk, [&] { return !writer && readers == 0; });
        --writers_waiting;
        writer = true;
    }
    void unlock() {
        std::lock_guard<std::mutex> lk(m);
        writer = false;
        cv.notify_all();
    }
};

}  // namespace

struct reann_server {
    Model *m = nullptr;
    reann_server_opts opt{};
    Ctx ctx;
    std::vector<double> minv;           // 1/mass per species (amu^-1), 0 = no dynamics
    DevBuf d_minv;
    std::mutex mu;                       // guards systems' registration, queue, results, stats
    std::condition_variable cv;
    std::map<uint64_t, std::unique_ptr<Sys>> systems;
    std::deque<Req> incoming;
    std::map<uint64_t, Done> results;
    std::map<uint64_t, bool> known;      // ticket -> outstanding
    uint64_t next_sys = 1, next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread engine;
    Slot slots[kSlots];
    std::list<Req> pending;              // engine-private
    // launcher pool: slots whose step is to be enqueued
    std::vector<std::thread> workers;
    std::mutex jmu;
    std::condition_variable jcv;
    std::deque<Slot *> jobs;
    bool wstop = false;                  // guarded by jmu
    // no capture on one thread overlaps an allocation or release on another; the steps that
    // only replay a graph and launch kernels take no lock
    CaptureGate gate;
    int64_t budget = 0, in_flight_atoms = 0;
    std::atomic<int64_t> resident{0};
    // test hook: the request with this ticket is refused as if its inputs were invalid
    // (environment variable REANN_SERVER_FAULT_TICKET at server creation; -1 = none)
    int64_t fault_ticket = -1;
    std::atomic<int64_t> stats[REANN_N_SERVER_STATS]{};
    std::string fatal;

    void run();
    void work();
    void enqueue(Slot &s);
    void reject(Slot &s);
    bool admit(Req &r);
    void finish(Slot &s);
    bool make_resident(Sys &sy, int64_t need);
    void evict(Sys &sy, bool copy_back = true);
    int64_t estimate_bytes(const Sys &sy) const;
    bool update_list(Slot &s, Sys &sy, bool list_valid, const double *h_pos, bool stale_known = false);
    void enqueue_tail(hipStream_t st, Sys &sy, bool vv, double dt, int32_t skip);
    void launch_tail(Slot &s, Sys &sy, bool vv, double dt, int32_t skip);
};

int64_t reann_server::estimate_bytes(const Sys &sy) const {
    // extended atoms: periodic images within r_c + skin of the box; pairs at the system density
    const double rc = m->r_c + opt.skin;
    double grow = 1.0, vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        const double L = sy.cell[4 * a];
        vol *= L > 0 ? L : 1.0;
        if (sy.pbc[a] && L > 0) grow *= 1.0 + 2.0 * rc / L;
    }
    const double n = (double)sy.n, ne = n * grow;
    const double dens = n / vol;
    const double pairs = std::max(1.0, n * dens * 4.18879 * rc * rc * rc) * 1.3 + ne * 8;
    const int K = m->K, NL = m->NL, F = m->F, H = m->H, nh = m->nh, T = opt.T;
    double b = 24 * ne + 4.0 * T * ne * K + 4.0 * T * n * NL * K + 4.0 * T * n * F + 8.0 * T * nh * n * H;
    b += 4.0 * n * (NL * K + F + 2 * std::max(F, H) + K + 4) + 4.0 * ne * (K + 3) + 8.0 * ne + 12.0 * pairs;
    b += 160.0 * n + 64.0 * ne;   // list bookkeeping, positions, velocities, forces
    return (int64_t)(b * 1.2) + (1 << 20);
}

void reann_server::evict(Sys &sy, bool copy_back) {
    std::shared_lock<CaptureGate> alloc(gate);
    // bring the evolving state home, then release the device memory
    if (sy.plan && copy_back) {
        // the system is idle: its last request's work is complete, so only these copies are waited for
        hipStream_t st = ctx.stream;
        HIP_OK(hipMemcpyAsync(sy.pos.data(), sy.d_pos.p, sy.n * 24, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(sy.vel.data(), sy.d_vel.p, sy.n * 24, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(sy.forces.data(), sy.d_Fold.p, sy.n * 24, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
    }
    sy.xref_ok = false;
    if (sy.tail) { (void)hipGraphExecDestroy(sy.tail); sy.tail = nullptr; }
    sy.free_host();
    sy.d_rng.release();
    sy.plan.reset();
    sy.d_pos.release(); sy.d_vel.release(); sy.d_Fold.release(); sy.d_out.release(); sy.d_aux.release();
    sy.d_spec.b.release();
    resident -= sy.bytes;
    sy.bytes = 0;
    stats[5] = resident.load();
}

bool reann_server::make_resident(Sys &sy, int64_t need) {
    if (resident + need > budget) {
        // evict idle systems, least recently used first
        std::vector<Sys *> idle;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &kv : systems)
                if (kv.second->plan && !kv.second->busy) idle.push_back(kv.second.get());
        }
        std::sort(idle.begin(), idle.end(), [](Sys *a, Sys *b) { return a->last_used < b->last_used; });
        for (Sys *v : idle) {
            if (resident + need <= budget) break;
            evict(*v);
        }
        if (resident + need > budget) return false;
    }
    std::shared_lock<CaptureGate> alloc(gate);
    hipStream_t st = ctx.stream;
    auto p = std::make_unique<Plan>();
    reann_opts o{};
    o.precision = opt.precision;
    o.skin = opt.skin;
    for (int a = 0; a < 3; ++a) o.decomp[a] = opt.decomp[a] > 0 ? opt.decomp[a] : 1;
    p->init(&ctx, m, sy.species.data(), sy.n, sy.cell, sy.pbc, opt.T, &o);
    sy.d_pos.ensure(sy.n * 24); sy.d_vel.ensure(sy.n * 24); sy.d_Fold.ensure(sy.n * 24);
    sy.d_out.ensure((kOutHead + 9 * sy.n) * 8);
    sy.d_aux.ensure((size_t)(kAuxKe + 3 * grid_for(sy.n * 3, kKeBlock)) * 8);
    sy.d_rng.ensure(16);
    sy.free_host();
    HIP_OK(hipHostMalloc((void **)&sy.h_res, (size_t)(kOutHead + 9 * sy.n) * 8, hipHostMallocDefault));
    HIP_OK(hipHostMalloc((void **)&sy.h_rng, 16, hipHostMallocDefault));
    sy.motion_known = sy.pred_known = false;
    int32_t *ds = sy.d_spec.resize(sy.n);
    HIP_OK(hipMemcpyAsync(ds, sy.species.data(), sy.n * 4, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(sy.d_pos.p, sy.pos.data(), sy.n * 24, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(sy.d_vel.p, sy.vel.data(), sy.n * 24, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(sy.d_Fold.p, sy.forces.data(), sy.n * 24, hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    sy.plan = std::move(p);
    sy.tail_rebuilds = -1;
    sy.bytes = need;   // corrected to the measured size after the first build
    resident += need;
    stats[5] = resident.load();
    return true;
}

// Neighbour-list upkeep of a step (positions already in place on the device; h_pos: the same
// positions on the host for EVAL requests).  The skin check on the device waits for the stream;
// it is skipped when the caller has shown the list valid (velocity-Verlet motion bounds), and
// for EVAL requests it runs on the host against the host copy of the positions the list was
// built from (the same rule: rebuild when an atom has moved more than skin/2).  stale_known: the
// caller has shown the list stale (a predicted drift), so it is rebuilt without a check.
// Returns whether the list was rebuilt.
bool reann_server::update_list(Slot &s, Sys &sy, bool list_valid, const double *h_pos, bool stale_known) {
    hipStream_t st = s.st;
    Plan &p = *sy.plan;
    if (!list_valid && h_pos && sy.xref_ok && p.built) {
        const double half = 0.5 * opt.skin;
        double d2max = 0.0;
        for (int64_t i = 0; i < sy.n; ++i) {
            const double dx = h_pos[3 * i] - sy.xref_h[3 * i], dy = h_pos[3 * i + 1] - sy.xref_h[3 * i + 1],
                         dz = h_pos[3 * i + 2] - sy.xref_h[3 * i + 2];
            d2max = std::max(d2max, dx * dx + dy * dy + dz * dz);
        }
        list_valid = d2max <= half * half;
    }
    // the device skin check (one wait for the stream) runs outside the gate, the rebuild inside
    bool stale = stale_known;
    if (!list_valid && !stale) {
        const int64_t tk = now_ns();
        stale = p.list_stale(sy.d_pos.as<double>(), st);
        stats[12]++;
        stats[13] += now_ns() - tk;
    }
    if (!stale) return false;
    {
        std::shared_lock<CaptureGate> alloc(gate);
        const int64_t tb = now_ns();
        p.rebuild(sy.d_pos.as<double>(), st, true);   // its last check is read when the step ends
        stats[10] += now_ns() - tb;
    }
    if (h_pos) {
        sy.xref_h.assign(h_pos, h_pos + 3 * sy.n);
        sy.xref_ok = true;
    } else {
        sy.xref_ok = false;
    }
    stats[6]++;
    const int64_t actual = (int64_t)p.device_bytes() + 4 * (int64_t)sy.n * 24;
    stats[5] = resident.fetch_add(actual - (int64_t)sy.bytes) + (actual - (int64_t)sy.bytes);
    sy.bytes = actual;
    return true;
}

// The step once the positions are in place: the forward and backward (E, F, W), then for a
// velocity-Verlet step the kick, the largest displacement since the list build, the kinetic
// energy and the thermostat (its draws read from d_rng), then the result vectors and the copy of
// the head and of the vectors not in `skip` to the system's pinned buffer.  Enqueued only (no
// synchronisation, no allocation).
void reann_server::enqueue_tail(hipStream_t st, Sys &sy, bool vv, double dt, int32_t skip) {
    Plan &p = *sy.plan;
    const int64_t n3 = sy.n * 3;
    const int B = 256;
    p.launch_forward(sy.d_pos.as<double>(), sy.E(), nullptr, st);
    p.backward(nullptr, sy.F(), sy.W(), st);
    // the squared displacements since the list build, now (head[11]) and after the next drift of
    // dt (head[14]), raised by k_vv_post as integer maxima
    unsigned long long *dmax = reinterpret_cast<unsigned long long *>(sy.d_out.as<double>() + 11);
    if (vv && n3 <= kKeOneBlock) {
        hipLaunchKernelGGL(k_vv_kick_ke_one, dim3(1), dim3(kKeBlock), 0, st, n3, dt, sy.d_spec.ptr(), d_minv.as<double>(),
                           sy.d_vel.as<double>(), sy.d_Fold.as<double>(), sy.F(), dmax, opt.thermostat_K,
                           opt.thermostat_tau_fs, (int)opt.thermostat, sy.d_rng.as<double>(), sy.d_aux.as<double>(),
                           sy.KE());
        LAUNCH_OK("k_vv_kick_ke_one");
    } else if (vv) {
        const int nb = grid_for(n3, kKeBlock);
        double *aux = sy.d_aux.as<double>();
        hipLaunchKernelGGL(k_vv_kick_ke, dim3(nb), dim3(kKeBlock), 0, st, n3, dt, sy.d_spec.ptr(), d_minv.as<double>(),
                           sy.d_vel.as<double>(), sy.d_Fold.as<double>(), sy.F(), aux + kAuxKe, dmax);
        LAUNCH_OK("k_vv_kick_ke");
        hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(kKeBlock), 0, st, sy.n, nb, dt, opt.thermostat_K,
                           opt.thermostat_tau_fs, (int)opt.thermostat, sy.d_rng.as<double>(), aux, sy.KE());
        LAUNCH_OK("k_ke_final");
    }
    hipLaunchKernelGGL(k_vv_post, dim3(grid_for(sy.n, B)), dim3(B), 0, st, sy.n, dt, sy.d_spec.ptr(),
                       d_minv.as<double>(), sy.F(), sy.d_Fold.as<double>(), sy.d_pos.as<double>(), sy.P(),
                       sy.d_vel.as<double>(), sy.V(), sy.d_aux.as<double>(), vv ? 1 : 0, p.nl.inv_perm.ptr(),
                       p.nl.xref.ptr(), dmax);
    LAUNCH_OK("k_vv_post");
    // the head, then each wanted vector, contiguous runs in one copy
    const int64_t seg[4] = {0, kOutHead, kOutHead + n3, kOutHead + 2 * n3};
    const int64_t end[4] = {kOutHead, kOutHead + n3, kOutHead + 2 * n3, kOutHead + 3 * n3};
    const bool want[4] = {true, !(skip & REANN_OUT_FORCES), !(skip & REANN_OUT_POSITIONS),
                          !(skip & REANN_OUT_VELOCITIES)};
    for (int k = 0; k < 4;) {
        if (!want[k]) { ++k; continue; }
        int e = k;
        while (e + 1 < 4 && want[e + 1]) ++e;
        HIP_OK(hipMemcpyAsync(sy.h_res + seg[k], sy.d_out.as<double>() + seg[k], (end[e] - seg[k]) * 8,
                              hipMemcpyDeviceToHost, st));
        k = e + 1;
    }
}

// enqueue_tail as one HIP-graph replay (use_graph): captured for the request kind, time step,
// vectors wanted and list build it was made for, and captured again when one of them changes.
void reann_server::launch_tail(Slot &s, Sys &sy, bool vv, double dt, int32_t skip) {
    hipStream_t st = s.st;
    if (!opt.use_graph) {
        enqueue_tail(st, sy, vv, dt, skip);
        return;
    }
    Plan &p = *sy.plan;
    if (!sy.tail || sy.tail_rebuilds != p.rebuilds || sy.tail_vv != vv || sy.tail_skip != skip ||
        (vv && sy.tail_dt != dt)) {
        std::unique_lock<CaptureGate> cap(gate);
        const int64_t tc = now_ns();
        if (sy.tail) { (void)hipGraphExecDestroy(sy.tail); sy.tail = nullptr; }
        hipGraph_t g = nullptr;
        HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_tail(st, sy, vv, dt, skip);
        } catch (...) {
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        HIP_OK(hipStreamEndCapture(st, &g));
        hipError_t e = hipGraphInstantiate(&sy.tail, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIP_OK(e);
        sy.tail_rebuilds = p.rebuilds;
        sy.tail_vv = vv;
        sy.tail_skip = skip;
        sy.tail_dt = dt;
        stats[11] += now_ns() - tc;
    }
    const int64_t t0 = now_ns();
    HIP_OK(hipGraphLaunch(sy.tail, st));
    stats[8] += now_ns() - t0;
    stats[3]++;
}

bool reann_server::admit(Req &r) {
    Sys *syp;
    {
        std::lock_guard<std::mutex> lk(mu);   // registration may insert concurrently
        syp = systems.at(r.sys).get();
    }
    Sys &sy = *syp;
    if (sy.busy) return false;
    if (!sy.failed.empty()) {
        Done d;
        d.status = REANN_E_STATE;
        d.error = "the system failed in an earlier request: " + sy.failed;
        d.t_submit = r.t_submit;
        d.t_done = now_ns();
        std::lock_guard<std::mutex> lk(mu);
        results[r.ticket] = std::move(d);
        return true;   // consumed
    }
    Slot *s = nullptr;
    for (auto &x : slots)
        if (!x.active) { s = &x; break; }
    if (!s) return false;
    if (in_flight_atoms > 0 && in_flight_atoms + sy.n > opt.max_batch_atoms) return false;
    if (!sy.plan) {
        const int64_t need = estimate_bytes(sy);
        if (need > budget) {
            Done d;
            d.status = REANN_E_CAPACITY;
            d.error = "system does not fit the server's HBM budget";
            d.t_submit = r.t_submit;
            d.t_done = now_ns();
            std::lock_guard<std::mutex> lk(mu);
            results[r.ticket] = std::move(d);
            return true;   // consumed
        }
        if (!make_resident(sy, need)) {
            stats[4]++;
            return false;
        }
    }
    sy.busy = true;
    sy.last_used = now_ns();
    s->active = true;
    s->sys = &sy;
    s->req = std::move(r);
    s->state.store(kQueued);
    in_flight_atoms += sy.n;
    {
        std::lock_guard<std::mutex> lk(jmu);
        jobs.push_back(s);
    }
    jcv.notify_one();
    return true;
}

// Launcher thread: enqueue the admitted step of each slot handed over by the engine.
void reann_server::work() {
    (void)hipSetDevice(ctx.device);
    for (;;) {
        Slot *s;
        {
            std::unique_lock<std::mutex> lk(jmu);
            jcv.wait(lk, [&] { return wstop || !jobs.empty(); });
            if (jobs.empty()) return;
            s = jobs.front();
            jobs.pop_front();
        }
        const int64_t t0 = now_ns();
        try {
            enqueue(*s);
            stats[7] += now_ns() - t0;
            s->state.store(kLaunched, std::memory_order_release);
        } catch (const Error &e) {
            s->err = e.what();
            s->err_code = e.code;
            const bool device = e.code == REANN_E_DEVICE || e.code == REANN_E_NOMEM;
            s->state.store(device ? kFailed : kRejected, std::memory_order_release);
        } catch (const std::exception &e) {
            s->err = e.what();
            s->err_code = REANN_E_DEVICE;
            s->state.store(kFailed, std::memory_order_release);
        }
    }
}

// A request its launcher refused for its inputs (an invalid configuration found by the list
// build, for instance): that request fails with the launcher's status, its system's device
// state is dropped without a copy back, and the server goes on serving the others.
void reann_server::reject(Slot &s) {
    Sys &sy = *s.sys;
    HIP_OK(hipStreamSynchronize(s.st));   // whatever the step enqueued before it stopped ends first
    sy.failed = s.err;
    evict(sy, false);
    Done d;
    d.status = s.err_code;
    d.error = s.err;
    d.t_submit = s.req.t_submit;
    d.t_done = now_ns();
    s.active = false;
    sy.busy = false;
    in_flight_atoms -= sy.n;
    std::lock_guard<std::mutex> lk(mu);
    results[s.req.ticket] = std::move(d);
}

void reann_server::enqueue(Slot &slot) {
    Slot *s = &slot;
    Sys &sy = *s->sys;
    Req &r = s->req;
    if (fault_ticket >= 0 && (int64_t)r.ticket == fault_ticket)
        fail(REANN_E_INVALID, "fault injected for this request (REANN_SERVER_FAULT_TICKET)");
    hipStream_t st = s->st;
    const int64_t n3 = sy.n * 3;
    const int B = 256;
    const bool vv = r.kind == REANN_REQ_VV_STEP;
    if (vv && !sy.have_forces) {
        // forces at the current positions first (once per system)
        update_list(*s, sy, false, nullptr);
        sy.plan->launch_forward(sy.d_pos.as<double>(), sy.E(), nullptr, st);
        sy.plan->backward(nullptr, sy.F(), sy.W(), st);
        hipLaunchKernelGGL(k_copy_d, dim3(grid_for(n3, B)), dim3(B), 0, st, n3, sy.F(), sy.d_Fold.as<double>());
        LAUNCH_OK("k_copy_d");
        sy.have_forces = true;
    }
    // After a velocity-Verlet step the previous step has already found the displacement this
    // drift gives when dt is unchanged: the list is then known valid or known stale, with no
    // check on the device.  With another dt the motion of the previous step bounds it: the drift
    // moves atom component c by v_c dt + a_c dt^2 / 2, so no atom gets further than
    // disp + sqrt(3) (dt max|v_c| + dt^2 max|a_c| / 2) from where the list was built.
    bool list_valid = false, stale_known = false;
    if (vv && sy.pred_known && r.dt == sy.pred_dt) {
        list_valid = sy.pred < 0.5 * opt.skin * (1.0 - 1e-9);
        stale_known = !list_valid;
        stats[14]++;
    } else if (vv && sy.motion_known) {
        const double bound = sy.disp + 1.7320508075688772 * (r.dt * sy.vmax + 0.5 * r.dt * r.dt * sy.amax);
        list_valid = bound < 0.5 * opt.skin * (1.0 - 1e-9);
    }
    if (vv) {
        hipLaunchKernelGGL(k_vv_drift, dim3(grid_for(n3, B)), dim3(B), 0, st, sy.n, r.dt, sy.d_spec.ptr(),
                           d_minv.as<double>(), sy.d_pos.as<double>(), sy.d_vel.as<double>(), sy.d_Fold.as<double>());
        LAUNCH_OK("k_vv_drift");
        // CSVR: one normal and one chi-square (N_f - 1 degrees of freedom) per step from the
        // system's stream, drawn when that thermostat is on (the kernel reads them only then).
        // The previous step of this system has completed, so its copy of h_rng has been made.
        if (opt.thermostat == REANN_THERMO_CSVR && opt.thermostat_K > 0.0 && opt.thermostat_tau_fs > 0.0) {
            std::normal_distribution<double> nd(0.0, 1.0);
            std::gamma_distribution<double> gd(0.5 * (3.0 * (double)sy.n - 1.0), 2.0);
            sy.h_rng[0] = nd(sy.rng);
            sy.h_rng[1] = sy.n * 3 > 1 ? gd(sy.rng) : 0.0;
            HIP_OK(hipMemcpyAsync(sy.d_rng.p, sy.h_rng, 16, hipMemcpyHostToDevice, st));
        }
    } else {
        HIP_OK(hipMemcpyAsync(sy.d_pos.p, r.pos.data(), sy.n * 24, hipMemcpyHostToDevice, st));
    }
    update_list(*s, sy, list_valid, vv ? nullptr : r.pos.data(), stale_known);
    launch_tail(*s, sy, vv, r.dt, r.skip);
    sy.have_forces = true;
    HIP_OK(hipEventRecord(s->ev, st));
}


void reann_server::finish(Slot &s) {
    Sys &sy = *s.sys;
    sy.plan->check_deferred();   // an inconsistent list is a device error: the server stops
    const int64_t n3 = sy.n * 3;
    Done d;
    d.energy = sy.h_res[0];
    std::memcpy(d.virial, sy.h_res + 1, 72);
    const bool vv = s.req.kind == REANN_REQ_VV_STEP;
    d.kinetic = vv ? sy.h_res[10] : 0.0;
    sy.motion_known = sy.pred_known = vv;
    if (vv) {
        sy.disp = std::sqrt(sy.h_res[11]);
        sy.vmax = sy.h_res[12];
        sy.amax = sy.h_res[13];
        sy.pred = std::sqrt(sy.h_res[14]);   // NaN (a blown-up system) reads as stale
        sy.pred_dt = s.req.dt;
    }
    d.skip = s.req.skip;
    if (!(d.skip & REANN_OUT_FORCES)) d.forces.assign(sy.h_res + kOutHead, sy.h_res + kOutHead + n3);
    if (!(d.skip & REANN_OUT_POSITIONS)) d.positions.assign(sy.h_res + kOutHead + n3, sy.h_res + kOutHead + 2 * n3);
    if (!(d.skip & REANN_OUT_VELOCITIES))
        d.velocities.assign(sy.h_res + kOutHead + 2 * n3, sy.h_res + kOutHead + 3 * n3);
    d.t_submit = s.req.t_submit;
    d.t_done = now_ns();
    sy.busy = false;
    in_flight_atoms -= sy.n;
    s.active = false;
    std::lock_guard<std::mutex> lk(mu);
    results[s.req.ticket] = std::move(d);
    stats[1]++;
    stats[2] += sy.n;
}

void reann_server::run() {
    try {
        HIP_OK(hipSetDevice(ctx.device));
        while (!stop.load()) {
            {
                std::unique_lock<std::mutex> lk(mu);
                bool any_active = false;
                for (auto &x : slots) any_active = any_active || x.active;
                if (incoming.empty() && pending.empty() && !any_active)
                    cv.wait_for(lk, std::chrono::milliseconds(2));
                while (!incoming.empty()) {
                    pending.push_back(std::move(incoming.front()));
                    incoming.pop_front();
                }
            }
            bool progressed = false;
            for (auto &x : slots) {
                if (!x.active) continue;
                const int stt = x.state.load(std::memory_order_acquire);
                if (stt == kFailed) throw Error(REANN_E_DEVICE, x.err);
                if (stt == kRejected) {
                    reject(x);
                    progressed = true;
                    continue;
                }
                if (stt == kLaunched && hipEventQuery(x.ev) == hipSuccess) {
                    const int64_t t0 = now_ns();
                    finish(x);
                    stats[9] += now_ns() - t0;
                    progressed = true;
                }
            }
            bool admitted = false;
            for (auto it = pending.begin(); it != pending.end();) {
                // nothing more can start while every slot is taken
                bool free_slot = false;
                for (auto &x : slots) free_slot = free_slot || !x.active;
                if (!free_slot) break;
                if (admit(*it)) {
                    it = pending.erase(it);
                    progressed = admitted = true;
                } else {
                    ++it;
                }
            }
            if (admitted) stats[0]++;
            if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        for (auto &x : slots)
            if (x.active) {
                int stt;
                while ((stt = x.state.load(std::memory_order_acquire)) == kQueued)
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
                if (stt == kFailed) throw Error(REANN_E_DEVICE, x.err);
                if (stt == kRejected) {
                    reject(x);
                    continue;
                }
                HIP_OK(hipEventSynchronize(x.ev));
                finish(x);
            }
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = e.what();
        // fail everything still queued so pollers do not wait forever
        for (auto &r : pending) {
            Done d;
            d.status = REANN_E_DEVICE;
            d.error = fatal;
            results[r.ticket] = std::move(d);
        }
        pending.clear();
        for (auto &x : slots)
            if (x.active) {
                Done d;
                d.status = REANN_E_DEVICE;
                d.error = fatal;
                results[x.req.ticket] = std::move(d);
                x.active = false;
            }
    }
}

template <class F> static reann_status serve_guard(F &&f) {
    try {
        f();
        return REANN_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return REANN_E_NOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return REANN_E_DEVICE;
    }
}

extern "C" {

reann_status reann_server_create(const reann_model *m, const reann_server_opts *o, reann_server **out) {
    return serve_guard([&] {
        if (!m || !o || !out) fail(REANN_E_INVALID, "NULL argument");
        if (o->T < 1 || o->T > m->impl.T_max) fail(REANN_E_INVALID, "T must be in [1, T_max]");
        if (!(o->skin >= 0) || !std::isfinite(o->skin)) fail(REANN_E_INVALID, "skin must be >= 0");
        if (o->precision < REANN_FP64 || o->precision > REANN_FP8) fail(REANN_E_INVALID, "unknown precision");
        if (o->precision == REANN_FP8 && m->impl.form != REANN_FORM_REANN)
            fail(REANN_E_UNSUPPORTED, "this message form runs in FP64, FP32 or BF16");
        if (!(o->thermostat_K >= 0) || !(o->thermostat_tau_fs >= 0) || !std::isfinite(o->thermostat_K) ||
            !std::isfinite(o->thermostat_tau_fs))
            fail(REANN_E_INVALID, "thermostat temperature and time constant must be finite and >= 0");
        int nd = 0;
        HIP_OK(hipGetDeviceCount(&nd));
        if (o->device < 0 || o->device >= nd) fail(REANN_E_INVALID, "device index out of range");
        for (int a = 0; a < 3; ++a)
            if (o->decomp[a] < 0 || o->decomp[a] > kMaxSplit) fail(REANN_E_INVALID, "decomp must be in [0, 16]");
        if (o->thermostat != REANN_THERMO_BERENDSEN && o->thermostat != REANN_THERMO_CSVR)
            fail(REANN_E_INVALID, "unknown thermostat");
        HIP_OK(hipSetDevice(o->device));
        auto s = std::make_unique<reann_server>();
        s->m = const_cast<Model *>(&m->impl);
        s->opt = *o;
        if (s->opt.max_batch_atoms <= 0) s->opt.max_batch_atoms = 262144;
        s->ctx.device = o->device;
        HIP_OK(hipStreamCreateWithFlags(&s->ctx.stream, hipStreamNonBlocking));
        s->ctx.own_stream = true;
        size_t fr = 0, tot = 0;
        HIP_OK(hipMemGetInfo(&fr, &tot));
        s->budget = o->hbm_budget_bytes > 0 ? o->hbm_budget_bytes : (int64_t)(fr / 4 * 3);
        for (auto &x : s->slots) {
            HIP_OK(hipStreamCreateWithFlags(&x.st, hipStreamNonBlocking));
            HIP_OK(hipEventCreateWithFlags(&x.ev, hipEventDisableTiming));
        }
        s->minv.assign(s->m->n_species, 0.0);
        s->d_minv.ensure(s->m->n_species * 8);
        HIP_OK(hipMemcpy(s->d_minv.p, s->minv.data(), s->m->n_species * 8, hipMemcpyHostToDevice));
        s->m->weights(o->device, s->ctx.stream);
        if (o->precision != REANN_FP64) {
            const OpType op = o->precision == REANN_BF16 ? OpType::BF16 : (o->precision == REANN_FP8 ? OpType::FP8 : OpType::F32);
            s->m->mfma(o->device, s->ctx.stream, false, op);
            s->m->mfma(o->device, s->ctx.stream, true, op);
        }
        if (const char *ft = std::getenv("REANN_SERVER_FAULT_TICKET")) s->fault_ticket = std::atoll(ft);
        reann_server *raw = s.release();
        for (int k = 0; k < kWorkers; ++k) raw->workers.emplace_back([raw] { raw->work(); });
        raw->engine = std::thread([raw] { raw->run(); });
        *out = raw;
    });
}

reann_status reann_server_set_masses(reann_server *s, const double *masses) {
    return serve_guard([&] {
        if (!s || !masses) fail(REANN_E_INVALID, "NULL argument");
        std::lock_guard<std::mutex> lk(s->mu);
        for (int k = 0; k < s->m->n_species; ++k) {
            if (!(masses[k] > 0) || !std::isfinite(masses[k])) fail(REANN_E_INVALID, "masses must be > 0");
            s->minv[k] = 1.0 / masses[k];
        }
        HIP_OK(hipSetDevice(s->ctx.device));
        HIP_OK(hipMemcpy(s->d_minv.p, s->minv.data(), s->m->n_species * 8, hipMemcpyHostToDevice));
    });
}

reann_status reann_system_add(reann_server *s, const int32_t *species, int64_t n, const double cell[9],
                              const int32_t pbc[3], const double *pos, const double *vel, uint64_t *sys_id) {
    return serve_guard([&] {
        if (!s || !species || !cell || !pbc || !pos || !sys_id) fail(REANN_E_INVALID, "NULL argument");
        if (n <= 0) fail(REANN_E_INVALID, "n must be > 0");
        for (int64_t i = 0; i < n; ++i)
            if (species[i] < 0 || species[i] >= s->m->n_species) fail(REANN_E_INVALID, "species out of range");
        for (int64_t i = 0; i < 3 * n; ++i)
            if (!std::isfinite(pos[i]) || (vel && !std::isfinite(vel[i]))) fail(REANN_E_INVALID, "non-finite input");
        Geom g{};
        geom_init(g, cell, pbc, s->opt.decomp, s->m->r_c, s->opt.skin);   // validates the cell and split
        auto sy = std::make_unique<Sys>();
        sy->n = n;
        sy->species.assign(species, species + n);
        std::memcpy(sy->cell, cell, sizeof sy->cell);
        std::memcpy(sy->pbc, pbc, sizeof sy->pbc);
        sy->pos.assign(pos, pos + 3 * n);
        sy->vel.assign(3 * n, 0.0);
        if (vel) sy->vel.assign(vel, vel + 3 * n);
        sy->forces.assign(3 * n, 0.0);
        if (s->estimate_bytes(*sy) > s->budget) fail(REANN_E_CAPACITY, "system larger than the server's HBM budget");
        std::lock_guard<std::mutex> lk(s->mu);
        sy->id = s->next_sys++;
        sy->rng.seed(s->opt.seed ^ (0x9E3779B97F4A7C15ull * sy->id));
        *sys_id = sy->id;
        s->systems[sy->id] = std::move(sy);
    });
}

reann_status reann_submit(reann_server *s, const reann_request *req, uint64_t *ticket) {
    return serve_guard([&] {
        if (!s || !req || !ticket) fail(REANN_E_INVALID, "NULL argument");
        Req r;
        r.t_submit = now_ns();
        r.sys = req->sys_id;
        r.kind = req->kind;
        r.dt = req->dt_fs;
        if (req->skip_outputs & ~(REANN_OUT_FORCES | REANN_OUT_POSITIONS | REANN_OUT_VELOCITIES))
            fail(REANN_E_INVALID, "unknown REANN_OUT_* bits in skip_outputs");
        r.skip = req->skip_outputs;
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->fatal.empty()) fail(REANN_E_DEVICE, s->fatal);
        auto it = s->systems.find(req->sys_id);
        if (it == s->systems.end()) fail(REANN_E_INVALID, "unknown system");
        if (r.kind == REANN_REQ_EVAL) {
            if (!req->pos) fail(REANN_E_INVALID, "EVAL needs positions");
            const int64_t n3 = it->second->n * 3;
            for (int64_t i = 0; i < n3; ++i)
                if (!std::isfinite(req->pos[i])) fail(REANN_E_INVALID, "non-finite positions");
            r.pos.assign(req->pos, req->pos + n3);
        } else if (r.kind == REANN_REQ_VV_STEP) {
            if (!(r.dt > 0) || !std::isfinite(r.dt)) fail(REANN_E_INVALID, "dt must be > 0");
            for (int k = 0; k < s->m->n_species; ++k)
                if (s->minv[k] == 0.0) fail(REANN_E_STATE, "set masses before VV_STEP requests");
        } else {
            fail(REANN_E_INVALID, "unknown request kind");
        }
        r.ticket = s->next_ticket++;
        *ticket = r.ticket;
        s->known[r.ticket] = true;
        s->incoming.push_back(std::move(r));
        s->cv.notify_one();
    });
}

reann_status reann_poll(reann_server *s, uint64_t ticket, reann_result *res) {
    if (!s || !res) return REANN_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return REANN_E_UNKNOWN_TICKET;
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return REANN_PENDING;
    Done &d = it->second;
    if (d.status == REANN_OK && ((res->forces && (d.skip & REANN_OUT_FORCES)) ||
                                 (res->positions && (d.skip & REANN_OUT_POSITIONS)) ||
                                 (res->velocities && (d.skip & REANN_OUT_VELOCITIES)))) {
        set_last_error("the result holds no vector that the request skipped (skip_outputs)");
        return REANN_E_INVALID;
    }
    res->status = d.status;
    res->energy = d.energy;
    std::memcpy(res->virial, d.virial, sizeof d.virial);
    if (res->forces && !d.forces.empty()) std::memcpy(res->forces, d.forces.data(), d.forces.size() * 8);
    if (res->positions && !d.positions.empty()) std::memcpy(res->positions, d.positions.data(), d.positions.size() * 8);
    if (res->velocities && !d.velocities.empty())
        std::memcpy(res->velocities, d.velocities.data(), d.velocities.size() * 8);
    res->t_submit_ns = d.t_submit;
    res->t_done_ns = d.t_done;
    res->kinetic = d.kinetic;
    const reann_status st = d.status;
    if (st != REANN_OK) set_last_error(d.error);
    s->results.erase(it);
    s->known.erase(ticket);
    return st;
}

reann_status reann_server_stats(reann_server *s, int64_t *st) {
    if (!s || !st) return REANN_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    for (int k = 0; k < REANN_N_SERVER_STATS; ++k) st[k] = s->stats[k].load();
    return REANN_OK;
}

void reann_server_destroy(reann_server *s) {
    if (!s) return;
    s->stop.store(true);
    s->cv.notify_all();
    if (s->engine.joinable()) s->engine.join();
    {
        std::lock_guard<std::mutex> lk(s->jmu);
        s->wstop = true;
    }
    s->jcv.notify_all();
    for (auto &w : s->workers)
        if (w.joinable()) w.join();
    (void)hipSetDevice(s->ctx.device);
    (void)hipDeviceSynchronize();
    s->systems.clear();
    for (auto &x : s->slots) {
        (void)hipEventDestroy(x.ev);
        (void)hipStreamDestroy(x.st);
    }
    (void)hipStreamDestroy(s->ctx.stream);
    delete s;
}

}  // extern "C"
