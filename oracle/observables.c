/* CPU oracle: per-event observables (section 4.1; thrust and Durham rates for
 * the e+e- workload).  Test infrastructure only.
 *
 * Layout of the 12 values per event:
 *   pp : 0 Z pT, 1 Z rapidity, 2 Z azimuth (0 with no transverse recoil),
 *        3 phi*, 4 number of anti-kT jets (R 0.4, pT > 5, |eta| < 5),
 *        5 leading-jet pT (|eta| < 5), 6 leading-jet eta (pT > 5),
 *        7 second-jet pT (|eta| < 5), 8 Delta R of the two leading jets (both
 *        cuts; -1 if fewer than two), 9 final-state partons, 10 sum of final
 *        momenta minus initial (largest component), 11 unused
 *   ee : 0 1 - thrust, 1 y23, 2 y34, 3 y45, 4 y56 (Durham, E scheme),
 *        9 final-state partons, 10 momentum imbalance, others 0
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_int.h"

#define NOBS 12
#define MAXP OR_MAXM

int or_n_obs(void) { return NOBS; }

static int is_parton(int pid) { return pid == 21 || (pid != 0 && abs(pid) <= 5); }

static double rap(const double* p) { return 0.5 * log((p[0] + p[3]) / (p[0] - p[3])); }
static double pseudo(const double* p) {
    double pt = sqrt(p[1] * p[1] + p[2] * p[2]);
    return asinh(p[3] / pt);
}

/* anti-kT (R) with E-scheme recombination; jets returned sorted by pT */
static int antikt(double (*ps)[4], int n, double R, double (*jets)[4]) {
    double (*q)[4] = malloc(sizeof(double[4]) * (n > 0 ? n : 1));
    int alive = n, nj = 0;
    memcpy(q, ps, sizeof(double[4]) * n);
    int* on = malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) on[i] = 1;
    while (alive > 0) {
        double best = INFINITY;
        int bi = -1, bj = -1;
        for (int i = 0; i < n; ++i) {
            if (!on[i]) continue;
            double pti2 = q[i][1] * q[i][1] + q[i][2] * q[i][2];
            double diB = 1.0 / pti2;
            if (diB < best) { best = diB; bi = i; bj = -1; }
            double yi = rap(q[i]), phii = atan2(q[i][2], q[i][1]);
            for (int j = i + 1; j < n; ++j) {
                if (!on[j]) continue;
                double ptj2 = q[j][1] * q[j][1] + q[j][2] * q[j][2];
                double dy = yi - rap(q[j]);
                double dphi = fabs(phii - atan2(q[j][2], q[j][1]));
                if (dphi > OR_PI) dphi = 2.0 * OR_PI - dphi;
                double dR2 = dy * dy + dphi * dphi;
                double dij = fmin(1.0 / pti2, 1.0 / ptj2) * dR2 / (R * R);
                if (dij < best) { best = dij; bi = i; bj = j; }
            }
        }
        if (bj < 0) {
            memcpy(jets[nj++], q[bi], sizeof(double[4]));
            on[bi] = 0;
        } else {
            for (int m = 0; m < 4; ++m) q[bi][m] += q[bj][m];
            on[bj] = 0;
        }
        alive -= 1;
    }
    /* sort by pT, descending (insertion sort) */
    for (int i = 1; i < nj; ++i) {
        double tmp[4];
        memcpy(tmp, jets[i], sizeof(tmp));
        double pti = tmp[1] * tmp[1] + tmp[2] * tmp[2];
        int j = i - 1;
        while (j >= 0 && jets[j][1] * jets[j][1] + jets[j][2] * jets[j][2] < pti) {
            memcpy(jets[j + 1], jets[j], sizeof(tmp));
            --j;
        }
        memcpy(jets[j + 1], tmp, sizeof(tmp));
    }
    free(q);
    free(on);
    return nj;
}

static double thrust(double (*ps)[4], int n) {
    double sum = 0.0;
    for (int i = 0; i < n; ++i) sum += sqrt(ps[i][1] * ps[i][1] + ps[i][2] * ps[i][2] + ps[i][3] * ps[i][3]);
    if (n < 2 || !(sum > 0.0)) return 1.0;
    double best = 0.0;
    if (n == 2) {
        double d[3] = {ps[0][1] - ps[1][1], ps[0][2] - ps[1][2], ps[0][3] - ps[1][3]};
        return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / sum;
    }
    /* the optimal hemisphere split is a plane through the origin that can be
     * turned until it contains two momenta: try every pair and their signs */
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double nv[3] = {ps[i][2] * ps[j][3] - ps[i][3] * ps[j][2],
                            ps[i][3] * ps[j][1] - ps[i][1] * ps[j][3],
                            ps[i][1] * ps[j][2] - ps[i][2] * ps[j][1]};
            double P[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < n; ++k) {
                if (k == i || k == j) continue;
                double d = ps[k][1] * nv[0] + ps[k][2] * nv[1] + ps[k][3] * nv[2];
                double sg = d >= 0.0 ? 1.0 : -1.0;
                for (int m = 0; m < 3; ++m) P[m] += sg * ps[k][m + 1];
            }
            for (int si = -1; si <= 1; si += 2)
                for (int sj = -1; sj <= 1; sj += 2) {
                    double Q[3];
                    for (int m = 0; m < 3; ++m) Q[m] = P[m] + si * ps[i][m + 1] + sj * ps[j][m + 1];
                    double v = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
                    if (v > best) best = v;
                }
        }
    return best / sum;
}

/* Durham clustering: y values at which k+1 jets become k (k = 2..5) */
static void durham(double (*ps)[4], int n, double* y) {
    double (*q)[4] = malloc(sizeof(double[4]) * (n > 0 ? n : 1));
    memcpy(q, ps, sizeof(double[4]) * n);
    int* on = malloc(sizeof(int) * (n > 0 ? n : 1));
    double Evis = 0.0;
    for (int i = 0; i < n; ++i) { on[i] = 1; Evis += q[i][0]; }
    for (int k = 0; k < 4; ++k) y[k] = 0.0;
    int alive = n;
    while (alive > 1) {
        double best = INFINITY;
        int bi = -1, bj = -1;
        for (int i = 0; i < n; ++i) {
            if (!on[i]) continue;
            double ai = sqrt(q[i][1] * q[i][1] + q[i][2] * q[i][2] + q[i][3] * q[i][3]);
            for (int j = i + 1; j < n; ++j) {
                if (!on[j]) continue;
                double aj = sqrt(q[j][1] * q[j][1] + q[j][2] * q[j][2] + q[j][3] * q[j][3]);
                double c = (q[i][1] * q[j][1] + q[i][2] * q[j][2] + q[i][3] * q[j][3]) / (ai * aj);
                double emin = fmin(q[i][0], q[j][0]);
                double yij = 2.0 * emin * emin * (1.0 - c) / (Evis * Evis);
                if (yij < best) { best = yij; bi = i; bj = j; }
            }
        }
        /* alive -> alive-1 jets happens at y_{alive-1, alive} */
        int k = alive - 1;
        if (k >= 2 && k <= 5) y[k - 2] = best;
        for (int m = 0; m < 4; ++m) q[bi][m] += q[bj][m];
        on[bj] = 0;
        alive -= 1;
    }
    free(q);
    free(on);
}

int or_observables(const or_state* s, const or_events* ev, int64_t n, double* obs) {
    double (*ps)[4] = malloc(sizeof(double[4]) * MAXP);
    double (*jets)[4] = malloc(sizeof(double[4]) * MAXP);
    for (int64_t e = 0; e < n; ++e) {
        double* o = obs + e * NOBS;
        for (int k = 0; k < NOBS; ++k) o[k] = 0.0;
        int np = 0, nn = ev->n[e];
        double lm[4] = {0, 0, 0, 0}, lp[4] = {0, 0, 0, 0}, bal[4] = {0, 0, 0, 0};
        for (int q = 0; q < nn; ++q) {
            int64_t k = (int64_t)q * ev->cap + e;
            double p[4] = {ev->E[k], ev->px[k], ev->py[k], ev->pz[k]};
            int st = ev->status[k];
            for (int m = 0; m < 4; ++m) bal[m] += st > 0 ? p[m] : -p[m];
            if (st <= 0) continue;
            if (ev->pid[k] == 11) memcpy(lm, p, sizeof(lm));
            else if (ev->pid[k] == -11) memcpy(lp, p, sizeof(lp));
            else if (is_parton(ev->pid[k]) && np < MAXP) memcpy(ps[np++], p, sizeof(p));
        }
        if (s->c.process == 0) bal[0] -= s->sqrtS;
        double imb = 0.0;
        for (int m = 0; m < 4; ++m) imb = fmax(imb, fabs(bal[m]));
        o[9] = np;
        o[10] = imb;
        if (s->c.process == 0) {
            o[0] = 1.0 - thrust(ps, np);
            double y[4];
            durham(ps, np, y);
            for (int k = 0; k < 4; ++k) o[1 + k] = y[k];
            continue;
        }
        double Z[4];
        for (int m = 0; m < 4; ++m) Z[m] = lm[m] + lp[m];
        double zpt = sqrt(Z[1] * Z[1] + Z[2] * Z[2]);
        o[0] = zpt;
        o[1] = rap(Z);
        o[2] = (Z[1] == 0.0 && Z[2] == 0.0) ? 0.0 : atan2(Z[2], Z[1]);
        double dphi = fabs(atan2(lm[2], lm[1]) - atan2(lp[2], lp[1]));
        if (dphi > OR_PI) dphi = 2.0 * OR_PI - dphi;
        double cth = tanh(0.5 * (pseudo(lm) - pseudo(lp)));
        o[3] = tan(0.5 * (OR_PI - dphi)) * sqrt(fmax(0.0, 1.0 - cth * cth));
        /* jets from partons with non-zero transverse momentum */
        int nq = 0;
        for (int i = 0; i < np; ++i)
            if (ps[i][1] * ps[i][1] + ps[i][2] * ps[i][2] > 1e-18 * s->S) memcpy(ps[nq++], ps[i], sizeof(double[4]));
        int nj = antikt(ps, nq, 0.4, jets);
        int njet = 0, n_eta = 0;
        double j1[4] = {0, 0, 0, 0}, j2[4] = {0, 0, 0, 0};
        double j1pt = 0.0, j2pt = 0.0, j1eta = 0.0;
        int have1 = 0;
        for (int k = 0; k < nj; ++k) {
            double pt = sqrt(jets[k][1] * jets[k][1] + jets[k][2] * jets[k][2]);
            double et = pseudo(jets[k]);
            if (fabs(et) < 5.0) {
                if (n_eta == 0) j1pt = pt;
                else if (n_eta == 1) j2pt = pt;
                n_eta++;
            }
            if (pt > 5.0 && !have1) { j1eta = et; have1 = 1; }
            if (pt > 5.0 && fabs(et) < 5.0) {
                if (njet == 0) memcpy(j1, jets[k], sizeof(j1));
                else if (njet == 1) memcpy(j2, jets[k], sizeof(j2));
                njet++;
            }
        }
        o[4] = njet;
        o[5] = j1pt;
        o[6] = j1eta;
        o[7] = j2pt;
        if (njet >= 2) {
            double dy = pseudo(j1) - pseudo(j2);
            double dp = fabs(atan2(j1[2], j1[1]) - atan2(j2[2], j2[1]));
            if (dp > OR_PI) dp = 2.0 * OR_PI - dp;
            o[8] = sqrt(dy * dy + dp * dp);
        } else {
            o[8] = -1.0;
        }
    }
    free(ps);
    free(jets);
    return 0;
}
