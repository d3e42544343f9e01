"""Independent vectorised numpy transcription of the two-component step, used
only to cross-check the C oracle on tiny lattices (array shifts instead of
node loops; same equations: Eqs. 1, 3-10, wall potentials, half-way
bounce-back).  Test infrastructure."""
import numpy as np
CX = np.array([0,1,0,-1,0,1,-1,-1,1]); CY = np.array([0,0,1,0,-1,1,1,-1,-1])
W = np.array([4/9]+[1/9]*4+[1/36]*4); OPP = np.array([0,3,4,1,2,7,8,5,6])
def _h3(i, T0):
    """Third-order Hermite tensor of velocity i (2 x 2 x 2)."""
    c = np.array([CX[i], CY[i]], dtype=np.float64); I = np.eye(2)
    return (np.einsum('a,b,c->abc', c, c, c) - T0 * (np.einsum('a,bc->abc', c, I) +
            np.einsum('b,ac->abc', c, I) + np.einsum('c,ab->abc', c, I)))
def run(f, mask, tau, G, rho_s, g, steps, periodic_y, dt=np.float64, reg3=False):
    """reg3: add the third-order Hermite projection of f - feq to the
    regularized part (w_i / (6 T0^3) H3_i : a3)."""
    f = f.astype(dt); w = W.astype(dt); cx = CX.astype(dt); cy = CY.astype(dt)
    ny, nx = mask.shape
    fl = mask.astype(bool)
    # neighbour fluid flags
    def shifted(a, dx, dy, fill):
        r = np.roll(np.roll(a, -dx, axis=-1), -dy, axis=-2) if periodic_y else None
        if periodic_y: return r
        r = np.roll(a, -dx, axis=-1)
        out = np.full_like(r, fill)
        if dy == 0: out[...] = r
        elif dy == 1: out[..., :-1, :] = r[..., 1:, :]
        else: out[..., 1:, :] = r[..., :-1, :]
        return out
    nb_fluid = [shifted(fl, CX[i], CY[i], False) for i in range(9)]
    T0 = dt(1/3)
    for t in range(steps):
        rho = f.sum(axis=1)  # [2,ny,nx]
        jx = np.einsum('i,sixy->sxy', cx, f); jy = np.einsum('i,sixy->sxy', cy, f)
        rt = np.where(fl, rho[0]+rho[1], 1)
        ux = (jx[0]+jx[1])/rt; uy = (jy[0]+jy[1])/rt
        nu = T0*(np.array(tau, dtype=dt)-dt(0.5))
        taum = (rho[0]*nu[0]+rho[1]*nu[1])/rt/T0 + dt(0.5)
        fnew = np.zeros_like(f)
        for s in range(2):
            b = 1-s
            Sx = np.zeros_like(rt); Sy = np.zeros_like(rt)
            for i in range(1,9):
                rb = np.where(nb_fluid[i], shifted(rho[b], CX[i], CY[i], 0), dt(rho_s[b]))
                Sx += w[i]*cx[i]*rb; Sy += w[i]*cy[i]*rb
            usx = ux + dt(G)*Sx + dt(g[0]); usy = uy + dt(G)*Sy + dt(g[1])
            def feq(vx, vy, i):
                cu = cx[i]*vx+cy[i]*vy; usq = vx*vx+vy*vy
                return rho[s]*w[i]*(1+3*cu+dt(4.5)*cu*cu-dt(1.5)*usq+dt(4.5)*cu*cu*cu-dt(4.5)*cu*usq)
            pxx = np.zeros_like(rt); pxy = np.zeros_like(rt); pyy = np.zeros_like(rt)
            a3 = np.zeros((2, 2, 2) + rt.shape)
            for i in range(9):
                rs = np.where(fl, rho[s], 1)
                d = f[s,i]-feq(jx[s]/rs,jy[s]/rs,i)  # species' own equilibrium
                pxx += cx[i]*cx[i]*d; pxy += cx[i]*cy[i]*d; pyy += cy[i]*cy[i]*d
                if reg3:
                    a3 += _h3(i, 1/3)[..., None, None] * d
            om = 1-1/taum
            for i in range(9):
                fneq = w[i]*dt(4.5)*((cx[i]*cx[i]-T0)*pxx+2*cx[i]*cy[i]*pxy+(cy[i]*cy[i]-T0)*pyy)
                if reg3:
                    fneq = fneq + w[i] * dt(4.5) * np.einsum('abc,abcyx->yx', _h3(i, 1/3), a3)
                fp = (feq(usx,usy,i) + om*fneq)*fl
                # stream
                dst = shifted(fp, -CX[i], -CY[i], 0)  # value arriving at x from x - c_i
                src_fluid = shifted(fl, -CX[i], -CY[i], False)
                # pull: f_i(x) = fp_i(x-c_i) if x-c_i fluid else fp_opp(x) ... handle below
                fnew[s,i] += np.where(src_fluid, dst, 0)
                # bounce: fp_i at x with x+c_i solid goes to opp(i) at x
                fnew[s,OPP[i]] += np.where(~nb_fluid[i], fp, 0)
        f = fnew*fl
    return f
