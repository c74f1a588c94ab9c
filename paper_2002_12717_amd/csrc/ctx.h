// Internal context of the G1-G2 library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "common.h"
#include "g1g2.h"

struct Regs {
    cd* g1 = nullptr;
    cd* g2 = nullptr;
};

// Hubbard model.  A context holds a batch of independent clusters (one for
// g1g2_init, n for g1g2_batch_init).  Per cluster, h0 per spin is stored as a
// real diagonal plus an ELL list of off-diagonal entries (row i: neighbours
// nbr[i][z] with values h0_{i,nbr}); the drive adds s(t) * x_i to the diagonal
// of both spins.  Registers concatenate the clusters: G1 blocks [2][ns][ns],
// G2 blocks [ns]^4.
struct ClusterDesc {
    int ns, zmax;
    int g1off;          // offset of the cluster's G1 block in a G1 register
    int nbroff;         // offset of its [2][ns][zmax] neighbour table
    int d0off;          // offset of its [2][ns] diagonal of h0
    int xoff;           // offset of its [ns] drive profile
    long long g2off;    // offset of its G2 block in a G2 register
    long long doff;     // TPH, GW, DSL: offset (in units of ns^3 pairs) of its diagonal tensors
    double U;
};

// One work-group's share of a stage: G2 elements [start, end) of a cluster
// (per-element kernel) or wave units [start, end) (row kernel), or
// (start < 0) the whole G1 update of the cluster.
struct WorkItem {
    int cluster;
    int start, end;
};

struct HubbardData {
    int ncl = 0;
    std::vector<ClusterDesc> hdesc;
    ClusterDesc* desc = nullptr;   // device copy
    WorkItem* work = nullptr;      // device work list
    int nwork = 0;
    bool rows = false;             // row stage kernel (every ns <= 64, <= 4 neighbours)
    bool realhop = false;          // every hopping (off-diagonal h0) is real
    bool slices = false;           // slice stage kernel (every selfenergy, on row-kernel clusters)
    bool row64 = false;            // slice kernel: every cluster has ns = 64 (a wave per G2 row)
    int slice_elems = 0;           // slice kernel: G2 elements of the longest item (its LDS stage)
    WorkItem* dwork = nullptr;     // TPH, GW, DSL: work list of the diagonal gather
    int ndwork = 0;
    cd* diag = nullptr;            // per cluster n_diag [ns]^3 gathered diagonal tensors
    long long diag_elems = 0;      // complex elements of diag (0: the closure gathers none)
    std::vector<int> chunk;        // elements of G2 per work-group, per cluster
    int* nbr = nullptr;            // concatenated neighbour tables
    cd* hop = nullptr;
    double* d0 = nullptr;
    double* xdrv = nullptr;
    std::vector<double> h_d0;
    std::vector<double> drive_c, drive_tc, drive_x;
    double drive_tau = 1.0;
    double drive_value(double t) const;
    bool has_drive() const { return !drive_c.empty(); }
};

// General basis: internal tensors are padded to nbp = roundup(nb, 16) so that
// every matrix-core tile is full; padding entries are kept exactly zero.
struct GeneralData {
    int nb = 0, nbp = 0;
    cd* h0 = nullptr;        // [nbp][nbp]
    cd* wm_rows = nullptr;   // W^- as pair matrix rows: [p][q][r][s] = w^-_pqrs   (nbp^4)
    cd* w_coll = nullptr;    // collision layout: [l][p][i][k] = w_iklp           (nbp^4)
    cd* w_hf = nullptr;      // mean-field layout: [i][j][l][k] = w^-_ikjl        (nbp^4)
    cd* vt = nullptr;        // scratch: transposed right sandwich                (nbp^4)
    cd* dmat = nullptr;      // scratch: D = T^dagger - R                         (nbp^4)
    cd* hhf = nullptr;       // scratch: h^HF of the current stage [nbp][nbp]
    cd* gg = nullptr;        // scratch: G^> of the current stage [nbp][nbp]
    cd* ipart = nullptr;     // scratch: collision-integral partial sums [nbp^2][nipart]
    int nipart = 0;
    // GW and the ladders: quasi-Hamiltonian and permuted G2 operand of a GEMM
    cd* heps = nullptr;      // GW: [(p,q)][(j,l)] = h^eps_qjpl; ladders: h^pp, h^ph (nbp^4)
    cd* bmat = nullptr;      // GW: [(i,k)][(p,q)] = G2_ipkq; ladders: see gen_bmat  (nbp^4)
    cd* pimat = nullptr;     // Pi_ijkl at [i][j][k][l], then at [l][k][j][i]       (2 nbp^4)
    cd* w_gw = nullptr;      // GW layout: [p][q][s][r] = w_sqrp                   (nbp^4)
    cd* w_pp = nullptr;      // TPP layout: [k][l][p][q] = w_pqkl                  (nbp^4)
    cd* w_ph = nullptr;      // TPH layout: [j][k][p][q] = w_pjkq                  (nbp^4)
    cd* icoll = nullptr;     // collision integral of the last RHS evaluation [nbp][nbp]
    // mixed precision copies of the constant layouts
    float2* wm_rows32 = nullptr;
    float2* w_coll32 = nullptr;
    float2* w_gw32 = nullptr;
    float2* w_pp32 = nullptr;
    float2* w_ph32 = nullptr;
};

// Jellium: momenta on a periodic grid; G1 [2][nb] (diagonal), G2 [3][nb]^3 in
// the momentum-transfer layout (jellium.hip).  sc/sb hold the partial sums of
// the polarization sums S of a G2 register: sets 0 and 1 alternate over the
// four stages of a step, set 2 serves single right-hand sides and observables.
struct JelliumData {
    int dims[3] = {1, 1, 1};
    int nb = 0;
    double* eps = nullptr;   // [2][nb] one-particle energies
    double* v = nullptr;     // [nb] pair interaction v_q (v_0 = 0)
    cd* hhf = nullptr;       // [2][nb] h^HF of the current stage input
    cd* stot = nullptr;      // [2][nb][nb] S^a_{P,Q} of the current stage input
    cd* skew = nullptr;      // [2][nb][nb] the same at [a][Pb][Q] = S^a_{Pb+Q,Q}
    cd* sc[3] = {};          // [3][nb][nb] per-block sums over the middle momentum
    cd* sb[3] = {};          // [nb][nb] down-spin sums of the up-down block
    int parity = 0;          // buffer set holding the sums of the next stage input
    // T-matrix closures: the ladder sums of the stage input [3][nb]^3, the
    // transform of v over the grid divided by nb [nb], the twiddles of the
    // three dimensions [Lx + Ly + Lz] and the index table of S - K [nb][nb]
    cd* lad = nullptr;
    cd* vhat = nullptr;
    cd* tw = nullptr;
    int* subt = nullptr;
};

struct g1g2_ctx {
    g1g2_desc d{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    double t = 0.0;
    int64_t step = 0;
    size_t n1 = 0, n2 = 0;     // internal element counts of G1 and G2
    Regs y, acc, s0, s1, io;   // RK4 registers; io = scratch for g1g2_rhs
    int* dflag = nullptr;      // divergence flag (device int)
    unsigned long long* ddiv = nullptr;   // [1 + clusters]: step counter and first diverged step (DivGuard)
    int nguard = 0;                       // clusters covered by ddiv
    double* dscratch = nullptr;  // small device scratch for reductions
    int nscratch = 0;
    HubbardData hub;
    GeneralData gen;
    JelliumData jel;
    // adiabatic switching of the interaction (U or w) by phi(t), a sin^2 ramp
    // from 0 at switch_t_on to 1 at switch_t_on + switch_tau; switch_tau = 0: off
    double switch_t_on = 0.0, switch_tau = 0.0;
    double switch_value(double t) const;
    bool has_switch() const { return switch_tau > 0.0; }
    void* adj = nullptr;       // adjoint state (adjoint.hip)
    // captured RK4 steps (replayed by g1g2_step_rk4 when the stream is not NULL)
    hipGraphExec_t graph = nullptr;
    double graph_dt = 0.0;
    int graph_steps = 0;
    bool graphs = true;
    // kernel timing (g1g2_profile_rhs): events recorded after every launch
    bool prof = false;
    std::vector<hipEvent_t> prof_ev;
    std::vector<const char*> prof_name;
    size_t prof_used = 0;
    std::vector<const char*> prof_kernels;   // distinct kernel names of the last profile
};

// The context's divergence guard (kernel argument).
inline DivGuard guard_of(const g1g2_ctx* c) { return DivGuard{c->dflag, c->ddiv}; }

// Record a timing event after the kernel `name` when profiling is active.
void prof_mark(g1g2_ctx* c, const char* name);

g1g2_status set_error(g1g2_ctx* c, g1g2_status s, const std::string& msg);

#define HIP_OK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return set_error((ctx), _e == hipErrorOutOfMemory ? G1G2_ENOMEM : G1G2_EDEVICE, \
                             std::string(#expr) + ": " + hipGetErrorString(_e));           \
    } while (0)

// ---- Hubbard basis (hubbard.hip)
// h0s[c] is the host h0 of cluster c ([2][ns][ns]); U[c] its interaction;
// chunk[c] (0 = default) the G2 elements per work-group.
g1g2_status hub_setup(g1g2_ctx* c, int ncl, const int* ns, const double* U, const cd* const* h0s,
                      const int* chunk);
void hub_free(g1g2_ctx* c);
// Whole RK4 steps of one small single-channel cluster in one persistent
// work-group (ns^4 <= 4096, binary64, no drive or ramp, no kernel flag).
// Whole RK4 steps of one small cluster (SOA, TPP or TPH, ns <= 7, no drive, no
// switching ramp, no per-launch profile) in one persistent work-group: whether
// the context qualifies, and nsteps steps of size dt on its state.
bool hub_persistent_ok(const g1g2_ctx* c);
g1g2_status hub_step_persistent(g1g2_ctx* c, double dt, int64_t nsteps);
// One RK4 stage (or a plain RHS evaluation, mode RK_RHS) of the Hubbard system;
// hub_stage_diag takes the buffer of the TPH/GW/DSL diagonal gathers
// (hub_diag_bytes) instead of the context's own.
g1g2_status hub_stage(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y,
                      const Regs& acc, const Regs& out, double cb, double cc);
g1g2_status hub_stage_diag(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y,
                           const Regs& acc, const Regs& out, double cb, double cc, cd* diag);
size_t hub_diag_bytes(const g1g2_ctx* c);
// The static device scratch of g1g2_rhs_noalloc on the context's device:
// looked up once per device at context set-up.
g1g2_status hub_noalloc_setup(g1g2_ctx* c);
g1g2_status hub_observables(g1g2_ctx* c, const Regs& s, double t, g1g2_obs* o);
g1g2_status hub_site_observables(g1g2_ctx* c, const Regs& s, double* nu, double* nd, double* docc);
g1g2_status hub_batch_observables(g1g2_ctx* c, const Regs& s, double t, g1g2_obs* o);

// ---- general basis (general.hip)
g1g2_status gen_setup(g1g2_ctx* c, const cd* h0_host, const cd* w_host);
g1g2_status gen_set_h0(g1g2_ctx* c, const cd* h0_host);
g1g2_status gen_stage(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y,
                      const Regs& acc, const Regs& out, double cb, double cc);
g1g2_status gen_observables(g1g2_ctx* c, const Regs& s, double t, g1g2_obs* o);
// layout conversions between the unpadded ABI layout and the padded internal one
g1g2_status gen_pad(g1g2_ctx* c, const cd* src_dev, cd* dst_dev, int rank);
g1g2_status gen_unpad(g1g2_ctx* c, const cd* src_dev, cd* dst_dev, int rank);
void gen_free(g1g2_ctx* c);

// ---- jellium (jellium.hip)
int jel_max_nb();
g1g2_status jel_setup(g1g2_ctx* c, const int* dims, const double* eps, const double* v);
void jel_free(g1g2_ctx* c);
// the state register y changed (init, set_state): recompute the sums of its G2
g1g2_status jel_state_changed(g1g2_ctx* c);
g1g2_status jel_stage(g1g2_ctx* c, int mode, const Regs& in, const Regs& y, const Regs& acc, const Regs& out,
                      double cb, double cc);
g1g2_status jel_observables(g1g2_ctx* c, const Regs& s, g1g2_obs* o);

// ---- adjoint (adjoint.hip)
void adj_free(g1g2_ctx* c);
