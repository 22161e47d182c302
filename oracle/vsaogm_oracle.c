/*
 * FP64 CPU oracle for VSA-OGM (Snyder, Capodieci, Gorsich, Parsa,
 * "Brain Inspired Probabilistic Occupancy Grid Mapping with Vector Symbolic
 * Architectures", arXiv 2408.09066).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant with the GPU library; both read the same seeded
 * inputs and nothing else.
 *
 * Everything here is a plain, slow, double-precision transcription of the
 * method's definitions, in the paper's order:
 *   - tile centres and nearest-tile assignment   (Sec. III-B, Algorithm 1)
 *   - fractional-power encoding of a 2-D point   (Sec. III-A eqs. for
 *     fractional binding with a length scale; Sec. III-B 2-D encoding eq.)
 *   - bundling into the memory 2*beta+psi        (eq. bundling, Algorithm 1)
 *   - memory normalisation                       (Sec. III-B eq. vector-normalization)
 *   - similarity = normalised memory . location  (Sec. III-B eq. loc-query)
 *   - per-class max normalisation and squaring   (Sec. III-B eq. non-linearities)
 *   - local Shannon entropy over a disk mask     (Algorithm 2, entropy and mask eqs.)
 *   - softmax, signed difference, threshold      (eqs. softmax, psd, classification)
 *   - multi-map fusion                           (Algorithm 3)
 *
 * Representation.  A real d-dimensional SSP is held as its length-D discrete
 * Fourier spectrum (forward transform unnormalised, inverse scaled by 1/D).
 * The axis vectors have unit-modulus spectra exp(i*theta_k) with a
 * conjugate-symmetric phase vector, so raising a spectrum to the power x/l is
 * exp(i*theta_k*x/l).  The caller passes Theta[k] = theta_k / l (rad per
 * metre), both axes, for every bin k = 0..D-1.  The spectrum of the point
 * (x, y) is then exp(i*(Theta[k][0]*x + Theta[k][1]*y)), the memory spectrum
 * is the sum of its points' spectra, and by Parseval
 *   ||w||^2      = (1/D) sum_k |W_k|^2
 *   w . phi(c)   = (1/D) Re sum_k conj(W_k) exp(i Theta[k].c).
 * All D bins are summed explicitly; no symmetry is exploited, and every
 * coordinate is in the world frame.
 *
 * Readings of points the paper leaves open (documented with the build):
 *   - tiles are numbered row-major, beta = ty*tiles_x + tx, 0-based, and the
 *     memory of tile beta and class psi (1 = occupied) has index 2*beta+psi;
 *   - the nearest tile is the argmin of the squared distance in double
 *     precision, the lowest index winning an exact tie; a grid cell queries
 *     the memory of its own nearest tile;
 *   - an all-zero memory has similarity 0 everywhere; a class whose maximum
 *     similarity is <= 0 has Q = 0 everywhere; 0*log 0 = 0; natural log;
 *   - the disk mask uses integer cell offsets, inclusive (dx^2+dy^2 <= r^2),
 *     and only neighbours inside the grid are summed;
 *   - a cell is occupied when OGM >= rho.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fused
 * multiply-add contraction, so the tile argmin rounds exactly as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* lay[4] = {x0, y0, x1, y1}: extent split into tiles[0] x tiles[1] equal tiles. */

/* Centre of tile beta (getTileCenters in Algorithm 1). */
void vo_tile_center(const double* lay, const int32_t* tiles, int32_t beta,
                    double* mx, double* my)
{
    int32_t tx = beta % tiles[0];
    int32_t ty = beta / tiles[0];
    double wx = (lay[2] - lay[0]) / (double)tiles[0];
    double wy = (lay[3] - lay[1]) / (double)tiles[1];
    *mx = lay[0] + ((double)tx + 0.5) * wx;
    *my = lay[1] + ((double)ty + 0.5) * wy;
}

/* beta = argmin_k ||gamma - mu_k|| (Algorithm 1); lowest index on exact ties. */
int32_t vo_assign_tile(const double* lay, const int32_t* tiles, double x, double y)
{
    int32_t ntiles = tiles[0] * tiles[1];
    int32_t best = 0;
    double best_d2 = INFINITY;
    for (int32_t b = 0; b < ntiles; ++b) {
        double mx, my;
        vo_tile_center(lay, tiles, b, &mx, &my);
        double dx = x - mx;
        double dy = y - my;
        double d2 = dx * dx + dy * dy;
        if (d2 < best_d2) { best_d2 = d2; best = b; }
    }
    return best;
}

void vo_assign_tiles(const double* lay, const int32_t* tiles, const double* xy,
                     int64_t n, int32_t* beta_out)
{
    for (int64_t i = 0; i < n; ++i)
        beta_out[i] = vo_assign_tile(lay, tiles, xy[2 * i], xy[2 * i + 1]);
}

/* Number of memory vectors: delta^n tiles times 2 classes (Sec. III-B). */
int64_t vo_num_memories(const int32_t* tiles) { return 2 * (int64_t)tiles[0] * tiles[1]; }

/*
 * Algorithm 1: for each point, find its tile and add its location vector
 * (2-D fractional binding) to memory 2*beta+psi.  omega is
 * [2R][D][2] (re, im), accumulated in place (memories persist across calls,
 * as successive point clouds keep bundling into them).  Returns the number of
 * points rejected because psi is not 0 or 1 (those are not bundled).
 */
int64_t vo_encode(int32_t D, const double* theta, const double* lay, const int32_t* tiles,
                  const float* xy, const uint8_t* label, int64_t n, double* omega)
{
    int64_t bad = 0;
    int32_t* key = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] > 1) { key[i] = -1; ++bad; continue; }
        int32_t beta = vo_assign_tile(lay, tiles, (double)xy[2 * i], (double)xy[2 * i + 1]);
        key[i] = 2 * beta + (int32_t)label[i];
    }
    /* bins are independent, so they are split across threads */
#pragma omp parallel for schedule(static)
    for (int32_t k = 0; k < D; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            if (key[i] < 0) continue;
            double x = (double)xy[2 * i], y = (double)xy[2 * i + 1];
            double ph = theta[2 * k] * x + theta[2 * k + 1] * y;
            double* w = omega + ((size_t)key[i] * D + k) * 2;
            w[0] += cos(ph);
            w[1] += sin(ph);
        }
    }
    free(key);
    return bad;
}

/* ||w|| of one memory from its spectrum (Parseval, inverse DFT scaled by 1/D). */
double vo_norm(int32_t D, const double* w)
{
    double s = 0.0;
    for (int32_t k = 0; k < D; ++k) s += w[2 * k] * w[2 * k] + w[2 * k + 1] * w[2 * k + 1];
    return sqrt(s / (double)D);
}

/* Real-space dot product (w/||w||) . phi(c), evaluated bin by bin. */
static double similarity_at(int32_t D, const double* theta, const double* w, double nrm,
                            double cx, double cy)
{
    if (nrm == 0.0) return 0.0;
    double s = 0.0;
    for (int32_t k = 0; k < D; ++k) {
        double ph = theta[2 * k] * cx + theta[2 * k + 1] * cy;
        s += w[2 * k] * cos(ph) + w[2 * k + 1] * sin(ph); /* Re(conj(W_k) e^{i ph}) */
    }
    return s / ((double)D * nrm);
}

/* grid[3] = {x0, y0, res}, cell (i, j) centre = (x0 + (i+0.5) res, y0 + (j+0.5) res). */
static void cell_center(const double* grid, int64_t i, int64_t j, double* cx, double* cy)
{
    *cx = grid[0] + ((double)i + 0.5) * grid[2];
    *cy = grid[1] + ((double)j + 0.5) * grid[2];
}

/*
 * Eq. loc-query over a matrix of query cells: P[psi][j][i] for every cell of
 * an nx x ny grid, each cell querying the memories of its own nearest tile.
 */
void vo_similarity(int32_t D, const double* theta, const double* lay, const int32_t* tiles,
                   const double* omega, const double* grid, int32_t nx, int32_t ny, double* P)
{
    int64_t nmem = vo_num_memories(tiles);
    double* nrm = (double*)malloc(sizeof(double) * (size_t)nmem);
    for (int64_t m = 0; m < nmem; ++m) nrm[m] = vo_norm(D, omega + (size_t)m * D * 2);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < (int64_t)nx * ny; ++c) {
        int64_t i = c % nx, j = c / nx;
        double cx, cy;
        cell_center(grid, i, j, &cx, &cy);
        int32_t beta = vo_assign_tile(lay, tiles, cx, cy);
        for (int32_t psi = 0; psi < 2; ++psi) {
            int32_t key = 2 * beta + psi;
            P[(size_t)psi * nx * ny + c] =
                similarity_at(D, theta, omega + (size_t)key * D * 2, nrm[key], cx, cy);
        }
    }
    free(nrm);
}

/* Same as vo_similarity for a list of flat cell indices (j*nx + i); P is [2][ncells]. */
void vo_similarity_cells(int32_t D, const double* theta, const double* lay, const int32_t* tiles,
                         const double* omega, const double* grid, int32_t nx,
                         const int64_t* cells, int64_t ncells, double* P)
{
    int64_t nmem = vo_num_memories(tiles);
    double* nrm = (double*)malloc(sizeof(double) * (size_t)nmem);
    for (int64_t m = 0; m < nmem; ++m) nrm[m] = vo_norm(D, omega + (size_t)m * D * 2);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < ncells; ++q) {
        int64_t i = cells[q] % nx, j = cells[q] / nx;
        double cx, cy;
        cell_center(grid, i, j, &cx, &cy);
        int32_t beta = vo_assign_tile(lay, tiles, cx, cy);
        for (int32_t psi = 0; psi < 2; ++psi) {
            int32_t key = 2 * beta + psi;
            P[(size_t)psi * ncells + q] =
                similarity_at(D, theta, omega + (size_t)key * D * 2, nrm[key], cx, cy);
        }
    }
    free(nrm);
}

/* Cells of the disk mask: integer offsets with dx^2 + dy^2 <= r^2. */
int64_t vo_disk_count(int32_t r)
{
    int64_t c = 0;
    for (int32_t dy = -r; dy <= r; ++dy)
        for (int32_t dx = -r; dx <= r; ++dx)
            if ((int64_t)dx * dx + (int64_t)dy * dy <= (int64_t)r * r) ++c;
    return c;
}

/* Entropy term of one cell: -Q log Q with Q = (P/m)^2 (eq. non-linearities). */
static double entropy_term(double p, double m)
{
    if (!(m > 0.0)) return 0.0;
    double q = (p / m) * (p / m);
    if (q == 0.0) return 0.0;
    return -q * log(q);
}

/* Local entropy of class map P at cell (i, j) with disk radius r (Algorithm 2). */
static double local_entropy(const double* P, double m, int32_t nx, int32_t ny,
                            int64_t i, int64_t j, int32_t r)
{
    double h = 0.0;
    for (int32_t dy = -r; dy <= r; ++dy) {
        for (int32_t dx = -r; dx <= r; ++dx) {
            if ((int64_t)dx * dx + (int64_t)dy * dy > (int64_t)r * r) continue;
            int64_t ii = i + dx, jj = j + dy;
            if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
            h += entropy_term(P[jj * nx + ii], m);
        }
    }
    return h;
}

/*
 * Decoding stages after similarity: per-class maximum over the whole map,
 * normalise and square, local entropy with radii r_occ (class 1) and r_emp
 * (class 0), softmax over the two entropies, probabilistic signed difference,
 * threshold rho.  P, H are [2][ny][nx]; m is [2]; ogm [ny][nx]; label [ny][nx].
 */
void vo_postprocess(const double* P, int32_t nx, int32_t ny, int32_t r_occ, int32_t r_emp,
                    double rho, double* m, double* H, double* ogm, uint8_t* label)
{
    int64_t nc = (int64_t)nx * ny;
    for (int32_t psi = 0; psi < 2; ++psi) {
        double mx = -INFINITY;
        for (int64_t c = 0; c < nc; ++c)
            if (P[psi * nc + c] > mx) mx = P[psi * nc + c];
        m[psi] = mx;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t i = c % nx, j = c / nx;
        double h0 = local_entropy(P, m[0], nx, ny, i, j, r_emp);
        double h1 = local_entropy(P + nc, m[1], nx, ny, i, j, r_occ);
        if (H) { H[c] = h0; H[nc + c] = h1; }
        double e0 = exp(h0), e1 = exp(h1);
        double pr1 = e1 / (e0 + e1);
        double pr0 = e0 / (e0 + e1);
        double o = pr1 - pr0;
        if (ogm) ogm[c] = o;
        if (label) label[c] = (o >= rho) ? 1 : 0;
    }
}

/*
 * The same stages at a list of cells, given the full class maps' maxima m[2]
 * and, for each listed cell, its (2r+1)^2 neighbourhood of similarity values
 * (nb is [ncells][2][2R+1][2R+1] with R = max(r_occ, r_emp); entries outside
 * the grid must be flagged by the validity mask valid[ncells][2R+1][2R+1]).
 * Used where the whole map is too large for the oracle.
 */
void vo_postprocess_cells(const double* nb, const uint8_t* valid, int64_t ncells,
                          int32_t r_occ, int32_t r_emp, const double* m, double rho,
                          double* H, double* ogm, uint8_t* label)
{
    int32_t R = r_occ > r_emp ? r_occ : r_emp;
    int32_t w = 2 * R + 1;
    for (int64_t q = 0; q < ncells; ++q) {
        double h[2] = {0.0, 0.0};
        for (int32_t psi = 0; psi < 2; ++psi) {
            int32_t r = psi ? r_occ : r_emp;
            for (int32_t dy = -r; dy <= r; ++dy)
                for (int32_t dx = -r; dx <= r; ++dx) {
                    if ((int64_t)dx * dx + (int64_t)dy * dy > (int64_t)r * r) continue;
                    size_t o = (size_t)(dy + R) * w + (dx + R);
                    if (!valid[(size_t)q * w * w + o]) continue;
                    h[psi] += entropy_term(nb[((size_t)q * 2 + psi) * w * w + o], m[psi]);
                }
        }
        if (H) { H[q] = h[0]; H[ncells + q] = h[1]; }
        double e0 = exp(h[0]), e1 = exp(h[1]);
        double o = e1 / (e0 + e1) - e0 / (e0 + e1);
        if (ogm) ogm[q] = o;
        if (label) label[q] = (o >= rho) ? 1 : 0;
    }
}

/*
 * The decoding ablation of Sec. IV-B (decoding methodology): the intermediate value before the
 * softmax is act(nl(n(P))) with toggles for the normalisation n(P) = P / max P (per class, over
 * the whole map), the non-linearity nl(Q) = Q^2, and the activation act, one of
 * 0 = local Shannon entropy over the disk of radius r_psi (Algorithm 2), 1 = ReLU, 2 = tanh,
 * 3 = sigmoid, applied per cell.  The two classes' values then go through the softmax, the
 * signed difference and the threshold as in the default decoding (normalise on, square on,
 * entropy).  Readings: with normalisation off the raw P is used; a class whose maximum is
 * <= 0 has n(P) = 0; the entropy term -Q ln Q is 0 for Q <= 0.
 */
static double ablation_value(double p, double m, int normalize, int square)
{
    double q = p;
    if (normalize) q = (m > 0.0) ? p / m : 0.0;
    if (square) q = q * q;
    return q;
}

void vo_postprocess_ex(const double* P, int32_t nx, int32_t ny, int32_t r_occ, int32_t r_emp,
                       double rho, int32_t normalize, int32_t square, int32_t act,
                       double* m, double* A, double* ogm, uint8_t* label)
{
    int64_t nc = (int64_t)nx * ny;
    for (int32_t psi = 0; psi < 2; ++psi) {
        double mx = -INFINITY;
        for (int64_t c = 0; c < nc; ++c)
            if (P[psi * nc + c] > mx) mx = P[psi * nc + c];
        m[psi] = mx;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t i = c % nx, j = c / nx;
        double a[2];
        for (int32_t psi = 0; psi < 2; ++psi) {
            const double* Pp = P + psi * nc;
            if (act == 0) {
                int32_t r = psi ? r_occ : r_emp;
                double h = 0.0;
                for (int32_t dy = -r; dy <= r; ++dy)
                    for (int32_t dx = -r; dx <= r; ++dx) {
                        if ((int64_t)dx * dx + (int64_t)dy * dy > (int64_t)r * r) continue;
                        int64_t ii = i + dx, jj = j + dy;
                        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
                        double q = ablation_value(Pp[jj * nx + ii], m[psi], normalize, square);
                        if (q > 0.0) h += -q * log(q);
                    }
                a[psi] = h;
            } else {
                double q = ablation_value(Pp[c], m[psi], normalize, square);
                if (act == 1) a[psi] = q > 0.0 ? q : 0.0;
                else if (act == 2) a[psi] = tanh(q);
                else a[psi] = 1.0 / (1.0 + exp(-q));
            }
        }
        if (A) { A[c] = a[0]; A[nc + c] = a[1]; }
        double e0 = exp(a[0]), e1 = exp(a[1]);
        double o = e1 / (e0 + e1) - e0 / (e0 + e1);
        if (ogm) ogm[c] = o;
        if (label) label[c] = (o >= rho) ? 1 : 0;
    }
}

/*
 * Algorithm 3 (multi-map fusion): agents that share axis vectors, classes and
 * tiling hold memories with the same indices; the global set starts empty and
 * each agent's memory j is added to global memory j (created as zero when
 * first seen).  present[a][j] != 0 marks memory j as held by agent a.
 * omegas is [n_agents][nmem][D][2]; out is [nmem][D][2], out_present [nmem].
 */
void vo_fuse(int32_t n_agents, int64_t nmem, int32_t D, const double* omegas,
             const uint8_t* present, double* out, uint8_t* out_present)
{
    memset(out_present, 0, (size_t)nmem);
    for (int32_t a = 0; a < n_agents; ++a) {
        for (int64_t j = 0; j < nmem; ++j) {
            if (!present[(size_t)a * nmem + j]) continue;
            const double* w = omegas + ((size_t)a * nmem + j) * D * 2;
            double* o = out + (size_t)j * D * 2;
            if (!out_present[j]) {
                for (int64_t k = 0; k < 2 * (int64_t)D; ++k) o[k] = 0.0;
                out_present[j] = 1;
            }
            for (int64_t k = 0; k < 2 * (int64_t)D; ++k) o[k] += w[k];
        }
    }
}

int32_t vo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Host threads the following oracle calls use (timing only; results do not depend on it). */
void vo_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * ---------------------------------------------------------------------------
 * Three dimensions (the 3-D extension named as future work in Sec. V; the
 * method of Sec. III with a third axis).  Readings: the fractional binding of
 * Sec. III-A takes one axis vector per dimension, so the spectrum of the point
 * (x, y, z) is exp(i*(Theta[k][0] x + Theta[k][1] y + Theta[k][2] z)); tiles
 * are delta_x x delta_y x delta_z boxes numbered beta = (tz*ty_n + ty)*tx_n + tx;
 * voxel centres are (x0 + (i+1/2) res, y0 + (j+1/2) res, z0 + (l+1/2) res); the
 * entropy mask is the ball of integer offsets dx^2 + dy^2 + dz^2 <= r^2.
 * Everything else (normalisation, maxima, squaring, entropy, softmax, signed
 * difference, threshold) is unchanged.  theta is [D][3], lay is
 * {x0, y0, z0, x1, y1, z1}, tiles is {tx_n, ty_n, tz_n}.
 * ---------------------------------------------------------------------------
 */
void vo3_tile_center(const double* lay, const int32_t* tiles, int32_t beta,
                     double* mx, double* my, double* mz)
{
    int32_t tx = beta % tiles[0];
    int32_t ty = (beta / tiles[0]) % tiles[1];
    int32_t tz = beta / (tiles[0] * tiles[1]);
    *mx = lay[0] + ((double)tx + 0.5) * ((lay[3] - lay[0]) / (double)tiles[0]);
    *my = lay[1] + ((double)ty + 0.5) * ((lay[4] - lay[1]) / (double)tiles[1]);
    *mz = lay[2] + ((double)tz + 0.5) * ((lay[5] - lay[2]) / (double)tiles[2]);
}

int32_t vo3_assign_tile(const double* lay, const int32_t* tiles, double x, double y, double z)
{
    int32_t n = tiles[0] * tiles[1] * tiles[2];
    int32_t best = 0;
    double best_d2 = INFINITY;
    for (int32_t b = 0; b < n; ++b) {
        double mx, my, mz;
        vo3_tile_center(lay, tiles, b, &mx, &my, &mz);
        double dx = x - mx, dy = y - my, dz = z - mz;
        double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < best_d2) { best_d2 = d2; best = b; }
    }
    return best;
}

void vo3_assign_tiles(const double* lay, const int32_t* tiles, const double* xyz, int64_t n,
                      int32_t* beta_out)
{
    for (int64_t i = 0; i < n; ++i)
        beta_out[i] = vo3_assign_tile(lay, tiles, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
}

/* Algorithm 1 in 3-D: omega [2R][D][2] accumulated in place; returns rejected labels. */
int64_t vo3_encode(int32_t D, const double* theta, const double* lay, const int32_t* tiles,
                   const float* xyz, const uint8_t* label, int64_t n, double* omega)
{
    int64_t bad = 0;
    int32_t* key = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] > 1) { key[i] = -1; ++bad; continue; }
        int32_t beta = vo3_assign_tile(lay, tiles, (double)xyz[3 * i], (double)xyz[3 * i + 1],
                                       (double)xyz[3 * i + 2]);
        key[i] = 2 * beta + (int32_t)label[i];
    }
#pragma omp parallel for schedule(static)
    for (int32_t k = 0; k < D; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            if (key[i] < 0) continue;
            double ph = theta[3 * k] * (double)xyz[3 * i] + theta[3 * k + 1] * (double)xyz[3 * i + 1] +
                        theta[3 * k + 2] * (double)xyz[3 * i + 2];
            double* w = omega + ((size_t)key[i] * D + k) * 2;
            w[0] += cos(ph);
            w[1] += sin(ph);
        }
    }
    free(key);
    return bad;
}

static double similarity3_at(int32_t D, const double* theta, const double* w, double nrm,
                             double cx, double cy, double cz)
{
    if (nrm == 0.0) return 0.0;
    double s = 0.0;
    for (int32_t k = 0; k < D; ++k) {
        double ph = theta[3 * k] * cx + theta[3 * k + 1] * cy + theta[3 * k + 2] * cz;
        s += w[2 * k] * cos(ph) + w[2 * k + 1] * sin(ph);
    }
    return s / ((double)D * nrm);
}

/* grid {x0, y0, z0, res}; voxels listed by flat index (l*ny + j)*nx + i; P is [2][ncells]. */
void vo3_similarity_cells(int32_t D, const double* theta, const double* lay, const int32_t* tiles,
                          const double* omega, const double* grid, int32_t nx, int32_t ny,
                          const int64_t* cells, int64_t ncells, double* P)
{
    int64_t nmem = 2 * (int64_t)tiles[0] * tiles[1] * tiles[2];
    double* nrm = (double*)malloc(sizeof(double) * (size_t)nmem);
    for (int64_t m = 0; m < nmem; ++m) nrm[m] = vo_norm(D, omega + (size_t)m * D * 2);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < ncells; ++q) {
        int64_t i = cells[q] % nx, j = (cells[q] / nx) % ny, l = cells[q] / ((int64_t)nx * ny);
        double cx = grid[0] + ((double)i + 0.5) * grid[3];
        double cy = grid[1] + ((double)j + 0.5) * grid[3];
        double cz = grid[2] + ((double)l + 0.5) * grid[3];
        int32_t beta = vo3_assign_tile(lay, tiles, cx, cy, cz);
        for (int32_t psi = 0; psi < 2; ++psi) {
            int32_t key = 2 * beta + psi;
            P[(size_t)psi * ncells + q] =
                similarity3_at(D, theta, omega + (size_t)key * D * 2, nrm[key], cx, cy, cz);
        }
    }
    free(nrm);
}

int64_t vo3_ball_count(int32_t r)
{
    int64_t c = 0;
    for (int32_t dz = -r; dz <= r; ++dz)
        for (int32_t dy = -r; dy <= r; ++dy)
            for (int32_t dx = -r; dx <= r; ++dx)
                if ((int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz <= (int64_t)r * r) ++c;
    return c;
}

static double local_entropy3(const double* P, double m, int32_t nx, int32_t ny, int32_t nz,
                             int64_t i, int64_t j, int64_t l, int32_t r)
{
    double h = 0.0;
    for (int32_t dz = -r; dz <= r; ++dz)
        for (int32_t dy = -r; dy <= r; ++dy)
            for (int32_t dx = -r; dx <= r; ++dx) {
                if ((int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz > (int64_t)r * r) continue;
                int64_t ii = i + dx, jj = j + dy, ll = l + dz;
                if (ii < 0 || jj < 0 || ll < 0 || ii >= nx || jj >= ny || ll >= nz) continue;
                h += entropy_term(P[(ll * ny + jj) * nx + ii], m);
            }
    return h;
}

/* Decoding stages after similarity over a whole volume; P, H are [2][nz][ny][nx]. */
void vo3_postprocess(const double* P, int32_t nx, int32_t ny, int32_t nz, int32_t r_occ,
                     int32_t r_emp, double rho, double* m, double* H, double* ogm, uint8_t* label)
{
    int64_t nc = (int64_t)nx * ny * nz;
    for (int32_t psi = 0; psi < 2; ++psi) {
        double mx = -INFINITY;
        for (int64_t c = 0; c < nc; ++c)
            if (P[psi * nc + c] > mx) mx = P[psi * nc + c];
        m[psi] = mx;
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t i = c % nx, j = (c / nx) % ny, l = c / ((int64_t)nx * ny);
        double h0 = local_entropy3(P, m[0], nx, ny, nz, i, j, l, r_emp);
        double h1 = local_entropy3(P + nc, m[1], nx, ny, nz, i, j, l, r_occ);
        if (H) { H[c] = h0; H[nc + c] = h1; }
        double e0 = exp(h0), e1 = exp(h1);
        double o = e1 / (e0 + e1) - e0 / (e0 + e1);
        if (ogm) ogm[c] = o;
        if (label) label[c] = (o >= rho) ? 1 : 0;
    }
}
