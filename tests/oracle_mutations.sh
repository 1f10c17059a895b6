#!/bin/bash
# Mutation check of the FP64 oracle (CPU only, not collected by pytest).
# Plants one mistake at a time in a scratch copy of the oracle's C sources
# (entries "file::sed-expression"; a bare expression means mf4d_oracle.c) and
# runs the oracle's pin tests on it; each mistake should make a pin fail.
# Usage: bash tests/oracle_mutations.sh   (from the repository root)
set -u
root=$(cd "$(dirname "$0")/.." && pwd)
muts=(
 's|R(y - 1, x - 1) += tp\[k\] / 4.0;|R(y - 1, x - 1) -= tp[k] / 4.0;|'
 's|const double rs2 = 1.0 / sqrt(2.0);|const double rs2 = 1.0;|'
 's|double f = 1.0 / sqrt(1.0 + sqrt(ux\[p\] \* ux\[p\] + uy\[p\] \* uy\[p\]));|double f = 1.0 / sqrt(1.0 + (ux[p] * ux[p] + uy[p] * uy[p]));|'
 's|mu\[2\] = 0.5 \* (mu\[0\] + mu\[1\]);|mu[2] = mu[0];|'
 's|double s2 = sigma \* sigma;|double s2 = sigma;|'
 's|if (mode == REF_RIDGE \&\& nt2 > 0.0) return 0.0;|if (mode == REF_RIDGE \&\& nt2 < 0.0) return 0.0;|'
 's|E\[c\]\[3\] = rs2 \* (e1\[k\] \* e2\[l\] - e2\[k\] \* e1\[l\]);|E[c][3] = rs2 * (e1[k] * e2[l] + e2[k] * e1[l]);|'
 's|mu\[3\] = 0.0;|mu[3] = 1.0;|'
 's|double c = c_param > 0.0 ? c_param : 0.5 \* smax;|double c = c_param > 0.0 ? c_param : smax;|'
 's|if (V\[s \* m + p\] > bv)|if (V[s * m + p] >= bv)|'
 's|tau\[i\] = 3.0 \* T / (2.0 \* (double)M \* ((double)n \* n + n) \* c \* c);|tau[i] = 3.0 * T / (2.0 * (double)M * ((double)n * n + n) * c);|'
 's|int p = 2 \* n;|int p = 2 * n + 1;|'
 's|for (int y = 1 + phase; y < H - 1; y += 3)|for (int y = 1 + phase; y < H; y += 3)|'
 's|if (uxy) uxy\[c\] = (V(ym, xm) + V(yp, xp) - V(yp, xm) - V(ym, xp)) / 4.0;|if (uxy) uxy[c] = (V(ym, xm) + V(yp, xp) - V(yp, xm) - V(ym, xp)) / 2.0;|'
 's|double theta = 0.5 \* atan2(2.0 \* b, a - d);|double theta = 0.5 * atan2(b, a - d);|'
 's|if (nu1 >= 0.0) mu\[0\] = 1.0;|if (nu1 > 0.1) mu[0] = 1.0;|'
 's|double F = hxx\[p\] \* hxx\[p\] + 2.0 \* hxy\[p\] \* hxy\[p\] + hyy\[p\] \* hyy\[p\];|double F = hxx[p] * hxx[p] + hxy[p] * hxy[p] + hyy[p] * hyy[p];|'
 's|for (int k = 0; k < 4; ++k) D\[5 \* k\] = g\[p\];|for (int k = 0; k < 4; k += 3) D[5 * k] = g[p];|'
 's|if (fabs(l2) > fabs(l1)) { ex\[p\] = -e1y; ey\[p\] = e1x; }|if (fabs(l2) < fabs(l1)) { ex[p] = -e1y; ey[p] = e1x; }|'
 's|return v >= 0.0 ? floor(v + 0.5) : -floor(-v + 0.5);|return floor(v + 0.5);|'
 's|if (!(vmax\[q\] >= theta)) break;|if (!(vmax[q] >= theta)) continue;|'
 's|if (d < bd) { bd = d; best = s; }|if (d <= bd) { bd = d; best = s; }|'
 's|for (int t = 1; t <= tmax; ++t) {|for (int t = 1; t < tmax; ++t) {|'
 'crease_oracle.c::s|return m < 0.0 ? 1 : -1;|return m > 0.0 ? 1 : -1;|'
 'crease_oracle.c::s|return m > 0.0 ? q <= 0.0 : q >= 0.0;|return m > 0.0 ? q >= 0.0 : q <= 0.0;|'
 'crease_oracle.c::s|double tt = dc\[a\] / (dc\[a\] - dc\[b\]);|double tt = 0.5;|'
 'crease_oracle.c::s|if (t > 1.0) t = 1.0;|if (t > 2.0) t = 2.0;|'
 'mf4d3d_oracle.c::s|out\[6 \* m + c\] = (v\[IX(z, ym, xm)\] + v\[IX(z, yp, xp)\] - v\[IX(z, yp, xm)\] - v\[IX(z, ym, xp)\]) / 4.0;|out[6 * m + c] = (v[IX(z, ym, xm)] + v[IX(z, yp, xp)] - v[IX(z, yp, xm)] - v[IX(z, ym, xp)]) / 2.0;|'
 'mf4d3d_oracle.c::s|double RB = fabs(n\[0\]) / sqrt(fabs(n\[1\] \* n\[2\]));|double RB = fabs(n[0]) / fabs(n[2]);|'
 'mf4d3d_oracle.c::s|double w = (i == j) ? mu\[i\] : 0.5 \* (mu\[i\] + mu\[j\]);|double w = (i == j) ? mu[i] : mu[i];|'
 'mf4d3d_oracle.c::s|const double rs2 = 1.0 / sqrt(2.0);|const double rs2 = 1.0;|'
 'mf4d3d_oracle.c::s|if (mode == RIDGE3 \&\& (n\[1\] > 0.0 \|\| n\[2\] > 0.0)) return 0.0;|if (mode == RIDGE3 \&\& (n[1] < 0.0 \|\| n[2] < 0.0)) return 0.0;|'
 'mf4d3d_oracle.c::s|double a = tp\[k == 0 ? 1 : 3\] / 4.0;|double a = tp[k == 0 ? 1 : 3] / 2.0;|'
 'mf4d3d_oracle.c::s|if (fabs(n\[j\]) < fabs(n\[i\]))|if (n[j] < n[i])|'
 'mf4d3d_oracle.c::s|double c = c_param > 0.0 ? c_param : 0.5 \* smax;|double c = c_param > 0.0 ? c_param : smax;|'
 'mf4d3d_oracle.c::s|double gn = sqrt(der\[p\] \* der\[p\] + der\[m + p\] \* der\[m + p\] + der\[2 \* m + p\] \* der\[2 \* m + p\]);|double gn = sqrt(der[p] * der[p] + der[m + p] * der[m + p]);|'
 'mf4d3d_oracle.c::s|R(z - 1, y, x) += tp\[8\]; R(z, y, x) -= 2.0 \* tp\[8\]; R(z + 1, y, x) += tp\[8\];|R(z - 1, y, x) += tp[8]; R(z, y, x) -= 2.0 * tp[8]; R(z + 1, y, x) += tp[4];|'
)
pins="tests/test_oracle_schedule.py tests/test_oracle_scalespace.py tests/test_oracle_tensor_operator.py tests/test_oracle_filter.py tests/test_oracle_ext.py tests/test_oracle_crease.py tests/test_oracle_3d.py"
i=0
for m in "${muts[@]}"; do
  i=$((i+1)); d=$(mktemp -d)
  cp -r "$root/oracle" "$root/tests" "$root/paper_1611_06906_amd" "$d/"
  rm -f "$d"/oracle/*.so
  f=mf4d_oracle.c; e=$m
  case "$m" in *.c::*) f=${m%%::*}; e=${m#*::};; esac
  sed -i "$e" "$d/oracle/$f"
  if cmp -s "$d/oracle/$f" "$root/oracle/$f"; then echo "MUT $i ($f): pattern did not apply"; rm -rf "$d"; continue; fi
  (cd "$d" && timeout 300 python -m pytest $pins -x -q -p no:cacheprovider > log 2>&1); rc=$?
  if [ $rc -eq 0 ]; then echo "MUT $i ($f): not caught"; else echo "MUT $i ($f): caught by $(grep -m1 -o 'FAILED [^ ]*' "$d/log")"; fi
  rm -rf "$d"
done
