// tuning.hip -- the measured launch table (tuned.inc, written by
// paper_2601_17979_amd/tune.py on the GPU) and its lookups, used by the
// plan when the caller leaves a choice open (nb = 0, inner_sweeps = 0,
// waves = 0).
#include "launchers.hpp"

namespace svdb {

namespace {

struct TunedBlock {
    int dtype;      // svdb_dtype_t; -1 ends the table
    int nmax;       // the class: n <= nmax ...
    int tall;       // ... and (m >= 2 n) == tall
    int nb;         // block width
    int inner;      // inner sweeps per block-pair solve (-1: converged)
    double tol_start, tol_rate;   // dynamic inner tolerance (tol_start 0: none)
};

struct TunedResident {
    int N, rw;      // padded columns and W rows per lane (0: packed); N -1 ends
    int waves;      // wavefronts per matrix
};

#include "tuned.inc"

}  // namespace

bool tuned_block(int dtype, int m, int n, BlockChoice *c)
{
    const int tall = m >= 2 * n;
    for (const TunedBlock &r : kTunedBlock) {
        if (r.dtype < 0) break;
        if (r.dtype == dtype && n <= r.nmax && r.tall == tall) {
            c->nb = r.nb;
            c->inner = r.inner;
            c->tol_start = r.tol_start;
            c->tol_rate = r.tol_rate;
            return true;
        }
    }
    return false;
}

int tuned_resident_waves(int N, int rw)
{
    for (const TunedResident &r : kTunedResident) {
        if (r.N < 0) break;
        if (r.N == N && r.rw == rw) return r.waves;
    }
    return 0;
}

}  // namespace svdb
